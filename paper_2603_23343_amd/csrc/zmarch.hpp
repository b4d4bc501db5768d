// zmarch.hpp -- the z-pencil streaming skeleton of every seven-point kernel.
//
// The paper (Sec. VI-A) gives each Tensix core a column of tiles: its x-y
// footprint over all z. Here a work-group owns a TX x TY footprint and a
// chunk of ZC planes and marches up z:
//   * z neighbours live in registers (planes k-1, k, k+1 of the thread's own
//     points), so each plane is read from HBM once;
//   * x/y neighbours come from a double-buffered LDS copy of plane k with a
//     one-point halo ring; halo rows/columns are loaded by a few threads and
//     mostly hit L2, since neighbouring tiles run on the same XCD;
//   * loads run D planes ahead of use through a register pipeline. Every
//     load is issued unconditionally (out-of-grid lanes read element 0 and
//     are zeroed when the value is consumed), so the compiler's wait for a
//     load lands where its value is used, D planes later, not at the load;
//   * points outside the grid read as 0 (zero Dirichlet ghosts, Sec. VII),
//     which replaces the paper's zero-fill pass.
// One __syncthreads per plane: a thread can only overwrite an LDS buffer two
// planes later, after every thread has passed the barrier of the plane in
// between.
//
// A kernel is the skeleton plus two functors:
//   Loader -- produces the values of the field the stencil is applied to
//             (a plain load, or p = D^-1 r + beta p_old computed on the fly,
//             halo included). fetch() issues loads into a raw register set,
//             finish() turns a raw set into compute-type values.
//   Op     -- fetch() issues the loads of the op's own streams for a plane;
//             apply() consumes, per thread and plane, those raw registers,
//             the centre values c[] and the stencil result ax[] of VX
//             consecutive points, and may accumulate NC reduction components.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace pcgmi {

// Tiles in x and y, z chunks of zc planes, nblocks = ntx * nty * nzc.
using Grid3 = Geometry;

template <typename C, int VX> struct Pts {
    C v[VX];
};

// N consecutive elements of T held as loaded (16-byte vector loads when the
// run is a whole number of 16-byte vectors, element loads otherwise).
template <typename T, int N, bool V = (N * sizeof(T) >= 16 && (N * sizeof(T)) % 16 == 0)> struct RawN;
template <typename T, int N> struct RawN<T, N, true> {
    static constexpr int W = 16 / (int)sizeof(T);
    static constexpr int NV = N / W;
    Vec16<T> v[NV];
    __device__ __forceinline__ void load(const T* p) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = reinterpret_cast<const Vec16<T>*>(p)[i];
    }
    // Non-temporal: the lines do not displace others in L2 and the last-level cache.
    __device__ __forceinline__ void load_nt(const T* p) {
        using U = __attribute__((__vector_size__(16))) unsigned int;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            U raw = __builtin_nontemporal_load(reinterpret_cast<const U*>(p) + i);
            __builtin_memcpy(&v[i], &raw, 16);
        }
    }
    __device__ __forceinline__ typename Traits<T>::C get(int i) const { return to_c(v[i / W].e[i % W]); }
};
template <typename T, int N> struct RawN<T, N, false> {
    T e[N];
    __device__ __forceinline__ void load(const T* p) {
#pragma unroll
        for (int i = 0; i < N; ++i) e[i] = p[i];
    }
    __device__ __forceinline__ void load_nt(const T* p) { load(p); }
    __device__ __forceinline__ typename Traits<T>::C get(int i) const { return to_c(e[i]); }
};

// ---------------------------------------------------------------------------
// Stencil policies. A policy names the per-point "cell" the skeleton stages in
// registers and LDS and the seven-point combination of a cell with its six
// face neighbours. Cells outside the grid are zero().
// ---------------------------------------------------------------------------

// Constant coefficients (paper Sec. VI/VII): (Ax)_p = 6 x_p - sum of the six neighbours.
template <typename C> struct StencilConst {
    using Cell = C;
    __device__ __forceinline__ static Cell zero() { return C(0); }
    __device__ __forceinline__ static C apply(const Cell& c, const Cell& l, const Cell& r, const Cell& d,
                                              const Cell& u, const Cell& b, const Cell& f) {
        return C(6) * c - l - r - d - u - b - f;
    }
};

// A field value with the cell coefficient k of its point.
template <typename C> struct UK {
    C u, k;
};

// Variable coefficients: (A_k u)_p = sum over faces of k_f (u_p - u_nb),
// k_f = 2 k_p k_q / (k_p + k_q) between cells p and q; on a boundary face
// (neighbour outside the grid, staged as k = 0) k_f = k_p and u_nb = 0.
template <typename C> struct StencilVar {
    using Cell = UK<C>;
    __device__ __forceinline__ static Cell zero() { return Cell{C(0), C(0)}; }
    __device__ __forceinline__ static C face(const Cell& c, const Cell& n) {
        const C kf = n.k == C(0) ? c.k : C(2) * c.k * n.k / (c.k + n.k);
        return kf * (c.u - n.u);
    }
    __device__ __forceinline__ static C apply(const Cell& c, const Cell& l, const Cell& r, const Cell& d,
                                              const Cell& u, const Cell& b, const Cell& f) {
        return face(c, l) + face(c, r) + face(c, d) + face(c, u) + face(c, b) + face(c, f);
    }
};

// Diagonal of the variable-coefficient operator: the sum of the six face
// coefficients (cells carry k only).
template <typename C> struct StencilVarDiag {
    using Cell = C;
    __device__ __forceinline__ static Cell zero() { return C(0); }
    __device__ __forceinline__ static C kf(C kc, C kn) { return kn == C(0) ? kc : C(2) * kc * kn / (kc + kn); }
    __device__ __forceinline__ static C apply(const Cell& c, const Cell& l, const Cell& r, const Cell& d,
                                              const Cell& u, const Cell& b, const Cell& f) {
        return kf(c, l) + kf(c, r) + kf(c, d) + kf(c, u) + kf(c, b) + kf(c, f);
    }
};

// The field value of a cell.
template <typename C> __device__ __forceinline__ C cell_u(const C& c) { return c; }
template <typename C> __device__ __forceinline__ C cell_u(const UK<C>& c) { return c.u; }

// LDS row pitch: interior starts at column PAD (16-byte aligned), left halo at
// PAD-1, right halo at PAD+TX.
template <typename Cell> struct LdsPad {
    static constexpr int PAD = sizeof(Cell) >= 16 ? 1 : 16 / (int)sizeof(Cell);
};

template <typename Cell, int BX, int BY, int VX> struct ZTile {
    static constexpr int TX = BX * VX, TY = BY, NT = BX * BY;
    static constexpr int PAD = LdsPad<Cell>::PAD;
    static constexpr int PITCH = TX + 2 * PAD;
    static constexpr int PLANE = (TY + 2) * PITCH;
    static_assert(2 * BX + 2 * TY <= NT, "not enough threads for the halo ring");
};

#ifndef PCGMI_ZM_DEPTH
#define PCGMI_ZM_DEPTH 2
#endif
constexpr int ZM_DEPTH = PCGMI_ZM_DEPTH;  // planes of look-ahead of every load

// Runs the z-march for logical tile `tile` with stencil policy SP. Returns the
// op's accumulators in acc. Rows are g.pitch elements apart. With LM (lane
// mask), vector lanes at x >= nx (row padding up to the pitch) read as 0 and
// their stencil result is 0, so padding that starts at 0 stays 0 under every
// op; without it the vector path needs nx % VX == 0.
template <typename C, class SP, int BX, int BY, int VX, int NC, bool LM = false, class Loader, class Op>
__device__ __forceinline__ void zmarch(const Grid3& g, unsigned tile, const Loader& ld, const Op& op,
                                       C (&acc)[NC], typename SP::Cell* lds /* 2 * ZTile::PLANE cells */) {
    using Cell = typename SP::Cell;
    using ZT = ZTile<Cell, BX, BY, VX>;
    using FRaw = typename Loader::template Raw<VX>;
    using ORaw = typename Op::Raw;
    constexpr int D = ZM_DEPTH;

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int bx = (int)(tile % (unsigned)g.ntx);
    const int by = (int)((tile / (unsigned)g.ntx) % (unsigned)g.nty);
    const int bz = (int)(tile / ((unsigned)g.ntx * (unsigned)g.nty));
    const int x0 = bx * ZT::TX, y0 = by * ZT::TY;
    const int z0 = bz * g.zc;
    const int z1 = min(z0 + g.zc, g.nz);
    const int64_t sy = g.pitch, sz = (int64_t)g.pitch * g.ny;

    const int xs = x0 + tx * VX, ys = y0 + ty;
    const bool own = (xs < g.nx) && (ys < g.ny);  // nx % VX == 0 on the vector path unless LM
    const int64_t col = (int64_t)ys * sy + xs;
    bool lane_ok[VX];
#pragma unroll
    for (int i = 0; i < VX; ++i) lane_ok[i] = !LM || xs + i < g.nx;

    // Halo duty: threads [0, 2BX) load one vector of the y-halo rows,
    // threads [2BX, 2BX + 2TY) the aligned vector holding one point of the
    // x-halo columns (left: last element of the vector before the tile,
    // right: first element of the vector after it), so every halo load is
    // the same 16-byte load and needs no branch.
    // LDS column of element e of the vector of thread column t. Eight 4-byte
    // cells per thread (16-bit storage) go as two halves, elements 0-3 at
    // 4t and 4-7 at TX/2 + 4t, so a wavefront's 16-byte LDS accesses cover
    // consecutive banks; stored whole at 8t they hit every other group of
    // four banks (measured: half of the wave-cycles of the 16-bit stencil
    // waited on LDS).
    constexpr bool SPLIT = VX == 8 && sizeof(Cell) == 4;
    auto lcol = [](int t, int e) { return SPLIT ? (e < 4 ? 4 * t + e : ZT::TX / 2 + 4 * t + e - 4) : VX * t + e; };
    int hkind = 0;  // 0 none, 1 y-row vector, 2 x-column point
    int hvx = 0, hy = 0, lds_off = 0, hsel = 0, hv_t = 0;
    bool hvalid = false;
    if (tid < 2 * BX) {
        hkind = 1;
        int row = tid < BX ? -1 : ZT::TY;
        int v = tid % BX;
        hvx = x0 + v * VX;
        hy = y0 + row;
        hvalid = hvx < g.nx && hy >= 0 && hy < g.ny;
        lds_off = (row + 1) * ZT::PITCH + ZT::PAD;
        hv_t = v;
    } else if (tid < 2 * BX + 2 * ZT::TY) {
        hkind = 2;
        int t = tid - 2 * BX;
        int side = t / ZT::TY, row = t % ZT::TY;
        const int hx = side == 0 ? x0 - 1 : x0 + ZT::TX;
        hvx = side == 0 ? x0 - VX : x0 + ZT::TX;
        hsel = side == 0 ? VX - 1 : 0;
        hy = y0 + row;
        hvalid = hx >= 0 && hx < g.nx && hy < g.ny;
        lds_off = (row + 1) * ZT::PITCH + (side == 0 ? ZT::PAD - 1 : ZT::PAD + ZT::TX);
    }
    const int64_t hcol = (int64_t)hy * sy + hvx;

    // fvalid/hval_ok: the point exists (else it reads as 0). Fetches also skip
    // planes the chunk never consumes (field planes above z1, halo and op
    // planes from z1 on); skipped and invalid lanes read element 0.
    auto fvalid = [&](int k) { return own && k >= 0 && k < g.nz; };
    auto hval_ok = [&](int k) { return hvalid && k >= 0 && k < g.nz; };
    auto fetch_plane = [&](int k, FRaw& r) {
        ld.template fetch<VX>((fvalid(k) && k <= z1) ? col + k * sz : 0, r);
    };
    auto fetch_halo = [&](int k, FRaw& r) {
        ld.template fetch<VX>((hval_ok(k) && k < z1) ? hcol + k * sz : 0, r);
    };
    auto finish_plane = [&](int k, const FRaw& r, Pts<Cell, VX>& out) {
        ld.template finish<VX>(r, out.v);
        const bool ok = fvalid(k);
#pragma unroll
        for (int i = 0; i < VX; ++i) out.v[i] = (ok && lane_ok[i]) ? out.v[i] : SP::zero();
    };
    auto finish_halo = [&](int k, const FRaw& r, Pts<Cell, VX>& out) {
        ld.template finish<VX>(r, out.v);
        const bool ok = hval_ok(k);
        if (hkind == 2) out.v[0] = hsel == 0 ? out.v[0] : out.v[VX - 1];
#pragma unroll
        for (int i = 0; i < VX; ++i) out.v[i] = ok ? out.v[i] : SP::zero();
    };
    auto fetch_op = [&](int k, ORaw& r) { op.fetch((fvalid(k) && k < z1) ? col + k * sz : 0, r); };

    // Pipeline with D slots (D planes of look-ahead). At the top of step k,
    // with s = (k - z0) mod D:
    //   zm, zcur, zp : values of planes k-1, k, k+1
    //   f[s]         : raw loads of plane k+2 (slot s+j holds plane k+2+j)
    //   hv           : halo values of plane k;  h[s]: raw halo of plane k+1
    //   o[s]         : raw op loads of plane k
    // A slot is consumed first and then refilled with the plane D steps on,
    // so no register of an in-flight load is ever copied (a copy would make
    // the compiler wait for the load). The loop is unrolled by D so slot
    // roles are static.
    Pts<Cell, VX> zm, zcur, zp, hv;
    FRaw f[D], h[D];
    ORaw o[D];
    {
        // every prologue load in flight before the first is used (128^3: 5.13 -> 4.98 ms per solve)
        FRaw t0, t1, t2, th;
        fetch_plane(z0 - 1, t0);
        fetch_plane(z0, t1);
        fetch_plane(z0 + 1, t2);
        fetch_halo(z0, th);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            fetch_plane(z0 + 2 + j, f[j]);
            fetch_halo(z0 + 1 + j, h[j]);
            fetch_op(z0 + j, o[j]);
        }
        finish_plane(z0 - 1, t0, zm);
        finish_plane(z0, t1, zcur);
        finish_plane(z0 + 1, t2, zp);
        finish_halo(z0, th, hv);
    }

#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = C(0);

    const int lrow = (ty + 1) * ZT::PITCH + ZT::PAD;  // start of this thread's row in LDS
    // x-neighbours of the vector's first and last elements
    const int lleft = tx == 0 ? -1 : lcol(tx - 1, VX - 1);
    const int lright = tx == BX - 1 ? ZT::TX : lcol(tx + 1, 0);
    auto step = [&](int k, FRaw& fs, FRaw& hs, ORaw& os) {
        Cell* buf = lds + ((k - z0) & 1) * ZT::PLANE;
        // Stage plane k: own points and halo.
#pragma unroll
        for (int i = 0; i < VX; ++i) buf[lrow + lcol(tx, i)] = zcur.v[i];
        if (hkind == 1) {
#pragma unroll
            for (int i = 0; i < VX; ++i) buf[lds_off + lcol(hv_t, i)] = hv.v[i];
        } else if (hkind == 2) {
            buf[lds_off] = hv.v[0];
        }
        // Consume this slot's field and halo loads, refill it D planes on.
        Pts<Cell, VX> znext, hnext;
        finish_plane(k + 2, fs, znext);
        fetch_plane(k + 2 + D, fs);
        finish_halo(k + 1, hs, hnext);
        fetch_halo(k + 1 + D, hs);
        __syncthreads();
        Pts<C, VX> ax;
        const Cell* up = buf + lrow + ZT::PITCH;
        const Cell* dn = buf + lrow - ZT::PITCH;
        const Cell left = buf[lrow + lleft], right = buf[lrow + lright];
#pragma unroll
        for (int i = 0; i < VX; ++i) {
            const Cell l = i == 0 ? left : zcur.v[i - 1];
            const Cell r = i == VX - 1 ? right : zcur.v[i + 1];
            ax.v[i] = SP::apply(zcur.v[i], l, r, dn[lcol(tx, i)], up[lcol(tx, i)], zm.v[i], zp.v[i]);
            if constexpr (LM) ax.v[i] = lane_ok[i] ? ax.v[i] : C(0);
        }
        if (own) op.apply(col + k * sz, os, zcur.v, ax.v, acc);
        fetch_op(k + D, os);
        zm = zcur;
        zcur = zp;
        zp = znext;
        hv = hnext;
    };
    for (int k = z0; k < z1; k += D) {
#pragma unroll
        for (int j = 0; j < D; ++j)
            if (k + j < z1) step(k + j, f[j], h[j], o[j]);
    }
}

}  // namespace pcgmi
