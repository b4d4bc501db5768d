// multigrid.hip -- geometric multigrid V-cycle, the preconditioner the paper
// names as future work (Sec. VIII), for the seven-point operator with
// constant or cell coefficients (FP32 vectors).
//
// Hierarchy: level l+1 halves every dimension of level l (a coarse cell is
// the union of 2 x 2 x 2 fine cells). Every level solves the UNSCALED
// seven-point system A[k_l] u = g_l (k_l = mean of the children's k); with
// the coarse spacing doubled this is the rediscretised operator 4^-l A[k_l]
// with its right-hand side scaled by 4^l, so the restriction of a residual r
// is g_(l+1) = P^T r / 2 (= 4 P^T r / 8).
//   prolongation P: per dimension 3/4 of the coarse cell holding the fine
//     cell and 1/4 of the coarse cell on its other side (0 outside);
//   smoother: damped Jacobi u <- u + omega D^-1 (g - A u);
//   V-cycle(l): u = 0; nu sweeps; r = g - A u; g_(l+1) = P^T r / 2;
//     e = V-cycle(l+1); u += P e; nu sweeps;  coarsest: u = A^-1 g with the
//     inverse formed on the host (FP64 Cholesky) and applied as a dense
//     product.
// Kernels: the sweeps and the residual are z-march kernels (the stencil's
// skeleton: z neighbours in registers, x/y halo through LDS); the first sweep
// from u = 0 is computed on the fly by the loader (u = omega D^-1 g, halo
// included) and fused with the next sweep or the residual. Restriction and
// prolongation are gather kernels (their reads of the other grid hit L2).
#include "zkernel.hpp"

namespace pcgmi {

namespace {

PCGMI_ZKERNEL(k_mg_smooth)
PCGMI_ZKERNEL(k_mg_residual)

// ---------------------------------------------------------------- loaders

// The stored iterate u of the level (constant coefficients).
using LoadMgU = LoadField<float>;
// The stored iterate with its cell coefficient.
using LoadMgUK = LoadUK<float>;

// The first sweep from u = 0, on the fly: u = omega D^-1 g (constant D = 6).
struct LoadMgStart {
    template <int N> using Raw = RawN<float, N>;
    const float* __restrict__ g;
    float wd;  // omega / 6
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const { r.load(g + i); }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, float* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = wd * r.get(v);
    }
};

// The same with a variable diagonal: u = omega dinv g, with k.
struct LoadMgStartVar {
    template <int N> struct Raw {
        RawN<float, N> g, d, k;
    };
    const float* __restrict__ g;
    const float* __restrict__ dinv;
    const float* __restrict__ kc;
    float omega;
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const {
        r.g.load(g + i);
        r.d.load(dinv + i);
        r.k.load(kc + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, UK<float>* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = UK<float>{omega * r.d.get(v) * r.g.get(v), r.k.get(v)};
    }
};

// ---------------------------------------------------------------- ops

// One damped-Jacobi sweep: out = u + omega D^-1 (g - A u) (u the cell).
template <int VX, bool VAR> struct OpMgSmooth {
    using C = float;
    struct Raw {
        RawN<float, VX> g;
        RawN<float, VAR ? VX : 1> d;
    };
    const float* __restrict__ g;
    const float* __restrict__ dinv;
    float* __restrict__ out;
    float wd;  // omega / 6 (constant coefficients) or omega
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const {
        raw.g.load(g + i);
        if constexpr (VAR) raw.d.load(dinv + i);
    }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C o[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const C w = VAR ? wd * raw.d.get(v) : wd;
            o[v] = cell_u(c[v]) + w * (raw.g.get(v) - ax[v]);
        }
        st_pts<float, VX>(out, i, o);
    }
};

// The residual r = g - A u; with STORE_U also the cell u (the on-the-fly
// first sweep) is stored.
template <int VX, bool STORE_U> struct OpMgResidual {
    using C = float;
    struct Raw {
        RawN<float, VX> g;
    };
    const float* __restrict__ g;
    float* __restrict__ r;
    float* __restrict__ u;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const { raw.g.load(g + i); }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C rv[VX], uv[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            uv[v] = cell_u(c[v]);
            rv[v] = raw.g.get(v) - ax[v];
        }
        st_pts<float, VX>(r, i, rv);
        if constexpr (STORE_U) st_pts<float, VX>(u, i, uv);
    }
};

// The fine level's last sweep fused with the flexible iteration's select
// step: z = u + omega D^-1 (g - A u) with g = r, plus z.q and z.r for
// FinFlexBeta (split grid reduction). After a switch to Jacobi (FLEX_JACOBI)
// it writes z = D^-1 r instead, as the select step would.
template <int VX, bool VAR> struct OpMgSmoothSelect {
    using C = float;
    struct Raw {
        RawN<float, VX> g, q;
        RawN<float, VAR ? VX : 1> d;
    };
    const float* __restrict__ g;
    const float* __restrict__ dinv;
    const float* __restrict__ q;
    float* __restrict__ out;
    const SolveState* st;
    float wd;  // omega / 6 (constant coefficients) or omega
    bool jac;
    __device__ void init() { jac = (st->flags & FLEX_JACOBI) != 0; }
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const {
        raw.g.load(g + i);
        raw.q.load(q + i);
        if constexpr (VAR) raw.d.load(dinv + i);
    }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C o[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const C gv = raw.g.get(v);
            const C dv = VAR ? raw.d.get(v) : C(1) / C(6);
            const C w = VAR ? wd * dv : wd;
            o[v] = jac ? dv * gv : cell_u(c[v]) + w * (gv - ax[v]);
            acc[0] += o[v] * raw.q.get(v);
            acc[1] += o[v] * gv;
        }
        st_pts<float, VX>(out, i, o);
    }
};

template <int FAM, class SP, int BX, int BY, int VX, class L, class O>
hipError_t run_mg(const Geometry& g, const L& ld, const O& op, const int* done, hipStream_t s) {
    if (g.nblocks == 0) return hipSuccess;
    const Red none{nullptr, nullptr, 0};
    if constexpr (FAM == 0)
        hipLaunchKernelGGL((k_mg_smooth<float, SP, BX, BY, VX, 1, 0u, false, L, O, FinNone>), dim3(g.nblocks),
                           dim3(BX * BY), 0, s, g, ld, op, FinNone{}, none, done, 0);
    else
        hipLaunchKernelGGL((k_mg_residual<float, SP, BX, BY, VX, 1, 0u, false, L, O, FinNone>), dim3(g.nblocks),
                           dim3(BX * BY), 0, s, g, ld, op, FinNone{}, none, done, 0);
    return hipGetLastError();
}

// The fused last sweep: a reducing z-march (two components) whose finishing
// step applies FinFlexBeta (a one-work-group kernel after it from 64
// work-groups on, else the last work-group).
template <class SP, int BX, int BY, int VX, class L, class O>
hipError_t run_mg_select(const Geometry& g, const L& ld, const O& op, const MgSelect& sel, const int* done,
                         hipStream_t s) {
    return run_zmarch<ZF_MG_SELECT, float, SP, BX, BY, VX, 2, 0u, true>(g, ld, op, FinFlexBeta{sel.st, false}, sel.red,
                                                                     done, s);
}

// ---------------------------------------------------------------- transfers

// Transfers launch one thread per coarse cell (restriction) or per four
// consecutive fine cells of a row (prolongation, when nx % 4 == 0; else per
// fine cell), on a 3-D grid: blockIdx.y and blockIdx.z are the row and the
// plane, so no index needs a division.
constexpr int TX = 64, TY = 4;  // threads per work-group: 64 along x, 4 rows

// g_c = P^T r / 2: each coarse cell gathers the 4 x 4 x 4 fine cells 2I-1 ..
// 2I+2 per dimension with 1-D weights (1/4, 3/4, 3/4, 1/4), those inside.
// V2 (nx % 4 == 0): two coarse cells 2t, 2t+1 per thread from one 16-byte
// load of fine 4t..4t+3 per row plus the two cells beside it.
template <bool V2>
__global__ void __launch_bounds__(TX* TY) k_mg_restrict(const float* __restrict__ r, int nx, int ny, int nz,
                                                       float* __restrict__ gc, const int* done) {
    if (*done) return;
    const int cx = nx / 2, cy = ny / 2;
    const int t = blockIdx.x * TX + threadIdx.x, J = blockIdx.y * TY + threadIdx.y, K = blockIdx.z;
    if constexpr (V2) {
        if (4 * t >= nx || J >= cy) return;
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int dz = 0; dz < 4; ++dz) {
            const int k = 2 * K - 1 + dz;
            if (k < 0 || k >= nz) continue;
            const float wz = (dz == 0 || dz == 3) ? 0.25f : 0.75f;
#pragma unroll
            for (int dy = 0; dy < 4; ++dy) {
                const int j = 2 * J - 1 + dy;
                if (j < 0 || j >= ny) continue;
                const float w = wz * ((dy == 0 || dy == 3) ? 0.25f : 0.75f);
                const float* row = r + ((int64_t)k * ny + j) * nx;
                const float4 v = *reinterpret_cast<const float4*>(row + 4 * t);
                const float lo = t > 0 ? row[4 * t - 1] : 0.f;
                const float hi = 4 * t + 4 < nx ? row[4 * t + 4] : 0.f;
                a0 += w * (0.25f * lo + 0.75f * v.x + 0.75f * v.y + 0.25f * v.z);
                a1 += w * (0.25f * v.y + 0.75f * v.z + 0.75f * v.w + 0.25f * hi);
            }
        }
        *reinterpret_cast<float2*>(gc + ((int64_t)K * cy + J) * cx + 2 * t) = make_float2(0.5f * a0, 0.5f * a1);
        return;
    }
    const int I = t;
    if (I >= cx || J >= cy) return;
    float acc = 0.f;
#pragma unroll
    for (int dz = 0; dz < 4; ++dz) {
        const int k = 2 * K - 1 + dz;
        if (k < 0 || k >= nz) continue;
        const float wz = (dz == 0 || dz == 3) ? 0.25f : 0.75f;
#pragma unroll
        for (int dy = 0; dy < 4; ++dy) {
            const int j = 2 * J - 1 + dy;
            if (j < 0 || j >= ny) continue;
            const float wy = (dy == 0 || dy == 3) ? 0.25f : 0.75f;
            const float* row = r + ((int64_t)k * ny + j) * nx;
            const float2 mid = *reinterpret_cast<const float2*>(row + 2 * I);  // fine 2I, 2I+1
            float s = 0.75f * (mid.x + mid.y);
            if (I > 0) s += 0.25f * row[2 * I - 1];
            if (2 * I + 2 < nx) s += 0.25f * row[2 * I + 2];
            acc += wz * wy * s;
        }
    }
    gc[((int64_t)K * cy + J) * cx + I] = 0.5f * acc;
}

// u += P e: per dimension a fine cell takes 3/4 of the coarse cell holding it
// and 1/4 of the coarse cell on its other side. V4: four fine cells
// 4t..4t+3 of a row per thread (float4 u), which need coarse x 2t-1 .. 2t+2.
template <bool V4>
__global__ void __launch_bounds__(TX* TY) k_mg_prolong(float* __restrict__ u, int nx, int ny, int nz,
                                                      const float* __restrict__ ec, const int* done) {
    if (*done) return;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const int t = blockIdx.x * TX + threadIdx.x, j = blockIdx.y * TY + threadIdx.y, k = blockIdx.z;
    if (j >= ny) return;
    const int J = j >> 1, K = k >> 1;
    const int Jo = (j & 1) ? J + 1 : J - 1, Ko = (k & 1) ? K + 1 : K - 1;
    const bool yo = Jo >= 0 && Jo < cy, zo = Ko >= 0 && Ko < cz;
    // the 2 x 2 coarse rows (J or Jo) x (K or Ko) with their y-z weights
    const float* rows[4];
    float wr[4];
    rows[0] = ec + ((int64_t)K * cy + J) * cx;
    wr[0] = 0.5625f;  // 3/4 * 3/4
    rows[1] = yo ? ec + ((int64_t)K * cy + Jo) * cx : nullptr;
    wr[1] = 0.1875f;
    rows[2] = zo ? ec + ((int64_t)Ko * cy + J) * cx : nullptr;
    wr[2] = 0.1875f;
    rows[3] = (yo && zo) ? ec + ((int64_t)Ko * cy + Jo) * cx : nullptr;
    wr[3] = 0.0625f;
    float* urow = u + ((int64_t)k * ny + j) * nx;
    if constexpr (V4) {
        if (4 * t >= nx) return;
        const int I = 2 * t;  // coarse cells of fine 4t..4t+3: I, I, I+1, I+1
        float f[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!rows[q]) continue;
            const float* er = rows[q];
            const float c0 = er[I], c1 = er[I + 1];
            const float cm = I > 0 ? er[I - 1] : 0.f;
            const float cp = I + 2 < cx ? er[I + 2] : 0.f;
            f[0] += wr[q] * (0.75f * c0 + 0.25f * cm);
            f[1] += wr[q] * (0.75f * c0 + 0.25f * c1);
            f[2] += wr[q] * (0.75f * c1 + 0.25f * c0);
            f[3] += wr[q] * (0.75f * c1 + 0.25f * cp);
        }
        float4 v = *reinterpret_cast<float4*>(urow + 4 * t);
        v.x += f[0];
        v.y += f[1];
        v.z += f[2];
        v.w += f[3];
        *reinterpret_cast<float4*>(urow + 4 * t) = v;
    } else {
        const int i = t;
        if (i >= nx) return;
        const int I = i >> 1, Io = (i & 1) ? I + 1 : I - 1;
        const bool xo = Io >= 0 && Io < cx;
        float f = 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!rows[q]) continue;
            f += wr[q] * (0.75f * rows[q][I] + (xo ? 0.25f * rows[q][Io] : 0.f));
        }
        urow[i] += f;
    }
}

// k_c = mean of the 8 children.
__global__ void __launch_bounds__(TX* TY) k_mg_coarsen_k(const float* __restrict__ kf, int nx, int ny, int nz,
                                                        float* __restrict__ kc) {
    const int cx = nx / 2, cy = ny / 2;
    const int I = blockIdx.x * TX + threadIdx.x, J = blockIdx.y * TY + threadIdx.y, K = blockIdx.z;
    if (I >= cx || J >= cy) return;
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
            const float* row = kf + ((int64_t)(2 * K + dz) * ny + 2 * J + dy) * nx + 2 * I;
            s += row[0] + row[1];
        }
    kc[((int64_t)K * cy + J) * cx + I] = 0.125f * s;
}

// Coarsest level: u = Ainv g (Ainv symmetric, m x m, FP32). One wavefront
// per row: lanes stride the row's columns (coalesced: a row of the symmetric
// inverse is its column), then a butterfly sum; 4 rows per work-group.
__global__ void __launch_bounds__(256) k_mg_dense(const float* __restrict__ ainv, const float* __restrict__ g,
                                                  float* __restrict__ u, int m, const int* done) {
    if (*done) return;
    const int lane = threadIdx.x & 63, row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const float* a = ainv + (int64_t)row * m;
    float acc = 0.f;
    for (int j = lane; j < m; j += 64) acc += a[j] * g[j];
    acc = wave_sum(acc);
    if (lane == 0) u[row] = acc;
}

dim3 grid_xyz(int threads_x, int ny, int nz) {
    return dim3((unsigned)((threads_x + TX - 1) / TX), (unsigned)((ny + TY - 1) / TY), (unsigned)nz);
}

// One z-march launch of a level: sweep (FAM 0) or residual (FAM 1), the
// iterate read from `u` or, when u == nullptr, formed on the fly as the
// first sweep from zero.
struct MgStep {
    const MgLevel& L;
    float omega;
    const int* done;
    hipStream_t s;

    // the last sweep of the fine level with the select step fused (u stored)
    hipError_t sweep_select(const float* g, const float* u, float* out, const MgSelect& sel) const {
        return dispatch_cfg<4>(L.plan.cfg, [&]<int BX, int BY, int VX>() -> hipError_t {
            if (L.k) {
                OpMgSmoothSelect<VX, true> op{g, L.dinv, sel.q, out, sel.st, omega, false};
                return run_mg_select<StencilVar<float>, BX, BY, VX>(L.geo, LoadMgUK{u, L.k}, op, sel, done, s);
            }
            OpMgSmoothSelect<VX, false> op{g, nullptr, sel.q, out, sel.st, omega / 6.f, false};
            return run_mg_select<StencilConst<float>, BX, BY, VX>(L.geo, LoadMgU{u}, op, sel, done, s);
        });
    }
    hipError_t sweep(const float* g, const float* u, float* out) const {
        return dispatch_cfg<4>(L.plan.cfg, [&]<int BX, int BY, int VX>() -> hipError_t {
            if (L.k) {
                OpMgSmooth<VX, true> op{g, L.dinv, out, omega};
                if (u) return run_mg<0, StencilVar<float>, BX, BY, VX>(L.geo, LoadMgUK{u, L.k}, op, done, s);
                return run_mg<0, StencilVar<float>, BX, BY, VX>(L.geo, LoadMgStartVar{g, L.dinv, L.k, omega}, op,
                                                                 done, s);
            }
            OpMgSmooth<VX, false> op{g, nullptr, out, omega / 6.f};
            if (u) return run_mg<0, StencilConst<float>, BX, BY, VX>(L.geo, LoadMgU{u}, op, done, s);
            return run_mg<0, StencilConst<float>, BX, BY, VX>(L.geo, LoadMgStart{g, omega / 6.f}, op, done, s);
        });
    }
    // r = g - A u; with u == nullptr the first sweep is formed on the fly and
    // stored to u_store.
    hipError_t residual(const float* g, const float* u, float* r, float* u_store) const {
        return dispatch_cfg<4>(L.plan.cfg, [&]<int BX, int BY, int VX>() -> hipError_t {
            if (L.k) {
                if (u) {
                    OpMgResidual<VX, false> op{g, r, nullptr};
                    return run_mg<1, StencilVar<float>, BX, BY, VX>(L.geo, LoadMgUK{u, L.k}, op, done, s);
                }
                OpMgResidual<VX, true> op{g, r, u_store};
                return run_mg<1, StencilVar<float>, BX, BY, VX>(L.geo, LoadMgStartVar{g, L.dinv, L.k, omega}, op,
                                                                 done, s);
            }
            if (u) {
                OpMgResidual<VX, false> op{g, r, nullptr};
                return run_mg<1, StencilConst<float>, BX, BY, VX>(L.geo, LoadMgU{u}, op, done, s);
            }
            OpMgResidual<VX, true> op{g, r, u_store};
            return run_mg<1, StencilConst<float>, BX, BY, VX>(L.geo, LoadMgStart{g, omega / 6.f}, op, done, s);
        });
    }
};

#define MGCHK(expr)                          \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

// V-cycle from level l with right-hand side g, result written to out; with
// sel (level 0 only) the last sweep also does the flexible select step.
hipError_t vcycle(const MgHierarchy& H, int l, const float* g, float* out, const int* done, hipStream_t s,
                  const MgSelect* sel) {
    const MgLevel& L = H.lv[l];
    if (l == H.nlev - 1) {
        hipLaunchKernelGGL(k_mg_dense, dim3((unsigned)((L.n + 3) / 4)), dim3(256), 0, s, H.ainv, g, out, (int)L.n,
                           done);
        return hipGetLastError();
    }
    const MgStep st{L, H.omega, done, s};
    const int nu = H.nu;
    // pre-smoothing: the first sweep is formed on the fly inside the next launch
    float* cur = L.u[0];
    if (nu == 1) {
        MGCHK(st.residual(g, nullptr, L.r, cur));
    } else {
        MGCHK(st.sweep(g, nullptr, cur));  // sweeps 1 and 2
        for (int k = 3; k <= nu; ++k) {
            float* nxt = cur == L.u[0] ? L.u[1] : L.u[0];
            MGCHK(st.sweep(g, cur, nxt));
            cur = nxt;
        }
        MGCHK(st.residual(g, cur, L.r, nullptr));
    }
    // coarse-grid correction
    const MgLevel& Lc = H.lv[l + 1];
    if (L.nx % 4 == 0)
        hipLaunchKernelGGL(k_mg_restrict<true>, grid_xyz(Lc.nx / 2, Lc.ny, Lc.nz), dim3(TX, TY), 0, s, L.r, L.nx, L.ny,
                           L.nz, Lc.g, done);
    else
        hipLaunchKernelGGL(k_mg_restrict<false>, grid_xyz(Lc.nx, Lc.ny, Lc.nz), dim3(TX, TY), 0, s, L.r, L.nx, L.ny,
                           L.nz, Lc.g, done);
    MGCHK(hipGetLastError());
    MGCHK(vcycle(H, l + 1, Lc.g, Lc.out, done, s, nullptr));
    if (L.nx % 4 == 0)
        hipLaunchKernelGGL(k_mg_prolong<true>, grid_xyz(L.nx / 4, L.ny, L.nz), dim3(TX, TY), 0, s, cur, L.nx, L.ny, L.nz,
                           Lc.out, done);
    else
        hipLaunchKernelGGL(k_mg_prolong<false>, grid_xyz(L.nx, L.ny, L.nz), dim3(TX, TY), 0, s, cur, L.nx, L.ny, L.nz,
                           Lc.out, done);
    MGCHK(hipGetLastError());
    // post-smoothing; the last sweep writes out
    for (int k = 1; k <= nu; ++k) {
        float* nxt = k == nu ? out : (cur == L.u[0] ? L.u[1] : L.u[0]);
        if (k == nu && sel) MGCHK(st.sweep_select(g, cur, nxt, *sel));
        else MGCHK(st.sweep(g, cur, nxt));
        cur = nxt;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_mg_vcycle(const MgHierarchy& H, const float* g, float* out, const int* done, hipStream_t s,
                           const MgSelect* sel) {
    if (H.nlev < 1 || (sel && H.nlev < 2)) return hipErrorInvalidValue;
    return vcycle(H, 0, g, out, done, s, sel);
}

hipError_t launch_mg_coarsen_k(const float* kf, int nx, int ny, int nz, float* kc, hipStream_t s) {
    if (nx < 2 || ny < 2 || nz < 2) return hipSuccess;
    hipLaunchKernelGGL(k_mg_coarsen_k, grid_xyz(nx / 2, ny / 2, nz / 2), dim3(TX, TY), 0, s, kf, nx, ny, nz, kc);
    return hipGetLastError();
}

}  // namespace pcgmi
