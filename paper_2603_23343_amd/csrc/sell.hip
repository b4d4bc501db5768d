// sell.hip -- SpMV of a general sparse matrix in sliced ELLPACK
// (SELL-C-sigma; Kreutzer, Hager, Wellein, Fehske, Bishop, SIAM J. Sci.
// Comput. 36(5), 2014), the storage of the GPU comparison system of the
// paper's Sec. VII-A, whose CG is built from norm, dot, axpy and SpMV.
//
// The layout is built on the host from compressed rows. On the device one
// wavefront owns one chunk of C = 64 rows, one lane per row: slot j of the
// chunk is a contiguous 256-byte run of column indices and one of values, so
// both streams load fully coalesced (non-temporal: each slot is read once per
// product), and the x gathers go through L2. The work-group -> chunk mapping
// is XCD-aware: each XCD walks a contiguous range of rows, so the x lines a
// row's neighbours share (for a grid operator, the planes above and below)
// stay in that XCD's L2.
//
// The same slot loop serves Jacobi-PCG on a stored SPD matrix
// (pcg_sell_solve): product with p.q, update, direction, each reducing pass
// followed by a one-work-group finisher, device-resident scalars, and batches
// of 16 iterations replayed from a captured HIP graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "pcgmi.h"

namespace pcgmi {
const char* set_error(pcg_status st, const char* msg);
}

using namespace pcgmi;

namespace {

// Device-resident scalars of a Jacobi-PCG solve on a stored matrix.
struct SellState {
    double rho;      // r.z of the current residual
    double sigma;    // p.Ap
    double alpha;    // rho / sigma
    double beta;     // rho_new / rho
    double rr;       // ||r||^2 from the recursion
    double bb;       // ||b||^2
    double tol2;     // (rtol ||b||)^2
    double true_rr;  // ||b - A x||^2 in FP64
    int iters;       // A p products
    int done;        // 0 running, 1 converged, 2 breakdown, 3 maxit reached
    int maxit;
    int x_owed;      // x still lacks the last update's alpha p (x advances every second update)
    double alpha_prev;  // alpha of the update before
};
// The direction of iteration k (k = iters + 1 while it is formed and used
// by the product, k = iters in the update and the next direction) lives in
// buffer k % 2 of the two p buffers.

}  // namespace

struct pcg_sell_s {
    int64_t nrows = 0, ncols = 0, nnz = 0, nchunks = 0, nslots = 0;
    int64_t* chunk_ptr = nullptr;  // device, nchunks + 1
    int32_t* col = nullptr;        // device, nslots
    float* val = nullptr;          // device, nslots
    int32_t* perm = nullptr;       // device, nrows (null when sigma = 1)
    hipStream_t stream = nullptr;
    // solver workspace (allocated by the first pcg_sell_solve)
    float *r = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr, *dinv = nullptr;
    double* part = nullptr;
    SellState* st = nullptr;
    int* bad = nullptr;
    int diag_state = 0;  // 0 not checked, 1 positive diagonal, -1 not
    // 16 iterations captured as one HIP graph (on a private stream), replayed
    // while the caller's x stays the same
    int use_graph = 1;
    int max_restarts = 3;  // FP64-residual restarts after the recursion has converged
    hipStream_t capture = nullptr;
    hipGraphExec_t batch = nullptr;
    const double* batch_x = nullptr;
};

namespace {

constexpr int SELL_C = 64;       // rows per chunk = wavefront width
constexpr int SELL_WAVES = 4;    // chunks per work-group
constexpr int SELL_UNROLL = 8;   // slots in flight per lane

pcg_status serr(pcg_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pcg_status serr(pcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(st, buf);
    return st;
}

template <bool PERM>
__global__ void __launch_bounds__(SELL_C * SELL_WAVES)
    k_sell_spmv(int64_t nrows, int64_t nchunks, const int64_t* __restrict__ chunk_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val, const int32_t* __restrict__ perm,
                const float* __restrict__ x, float* __restrict__ y) {
    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t c = (int64_t)b * SELL_WAVES + (threadIdx.x >> 6);
    if (c >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const int64_t base = chunk_ptr[c];
    const int w = (int)((chunk_ptr[c + 1] - base) / SELL_C);
    const int32_t* cp = col + base + lane;
    const float* vp = val + base + lane;
    float acc = 0.0f;
    for (int j = 0; j < w; j += SELL_UNROLL) {
        int ci[SELL_UNROLL];
        float vi[SELL_UNROLL], xv[SELL_UNROLL];
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) {
            ci[u] = -1;
            vi[u] = 0.0f;
            if (j + u < w) {
                ci[u] = __builtin_nontemporal_load(cp + (int64_t)(j + u) * SELL_C);
                vi[u] = __builtin_nontemporal_load(vp + (int64_t)(j + u) * SELL_C);
            }
        }
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) xv[u] = ci[u] >= 0 ? x[ci[u]] : 0.0f;
        // entries in storage order; padding (column -1) is skipped
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u)
            if (ci[u] >= 0) acc = __builtin_fmaf(vi[u], xv[u], acc);
    }
    const int64_t s = c * SELL_C + lane;
    if (s < nrows) {
        const int64_t dst = PERM ? (int64_t)perm[s] : s;
        __builtin_nontemporal_store(acc, y + dst);
    }
}

// ---------------------------------------------------------------------------
// Jacobi-PCG on the stored matrix (the Hestenes-Stiefel form, Saad Alg. 9.1
// with M = D): per iteration q = A p with p.q (sliced-ELLPACK kernel), the
// update x += alpha p, r -= alpha q with r.r and r.z, and the direction
// p = D^-1 r + beta p. Each reducing kernel leaves one partial per
// work-group (fixed grid, contiguous ranges); a one-work-group finisher sums
// them in index order and updates the device state; every kernel returns at
// once when the state says the solve has ended, so the host can enqueue
// iterations in batches.
// ---------------------------------------------------------------------------
constexpr int SNT = 256;
constexpr unsigned SELL_MAX_GRID = 2048;    // streaming kernels
constexpr unsigned SELL_MAX_QGRID = 16384;  // product kernels (one to four chunks per wavefront at 256^3)
constexpr int FNT = 1024;                   // finisher threads for more than 4096 partials, else SNT
enum : int { FIN_START = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_TRUE = 3 };

__device__ __forceinline__ void block_range(int64_t n, int64_t& lo, int64_t& hi, unsigned& b) {
    b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    lo = (int64_t)b * per;
    hi = lo + per < n ? lo + per : n;
}

// The row at sorted position s of chunk c (lane = s mod 64): the sum of
// val * v[col] in storage order with fused multiply-adds in type A (FP32 as
// k_sell_spmv, or FP64).
template <typename V, typename A>
__device__ __forceinline__ A sell_row(const int64_t* __restrict__ chunk_ptr, const int32_t* __restrict__ col,
                                      const float* __restrict__ val, const V* __restrict__ v, int64_t c, int lane) {
    const int64_t base = chunk_ptr[c];
    const int w = (int)((chunk_ptr[c + 1] - base) / SELL_C);
    const int32_t* cp = col + base + lane;
    const float* vp = val + base + lane;
    A acc = A(0);
    for (int j = 0; j < w; j += SELL_UNROLL) {
        int ci[SELL_UNROLL];
        float vi[SELL_UNROLL];
        V xv[SELL_UNROLL];
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) {
            ci[u] = -1;
            vi[u] = 0.0f;
            if (j + u < w) {
                ci[u] = __builtin_nontemporal_load(cp + (int64_t)(j + u) * SELL_C);
                vi[u] = __builtin_nontemporal_load(vp + (int64_t)(j + u) * SELL_C);
            }
        }
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) xv[u] = ci[u] >= 0 ? v[ci[u]] : V(0);
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u)
            if (ci[u] >= 0) {
                if constexpr (sizeof(A) == 4) acc = __builtin_fmaf(vi[u], (float)xv[u], acc);
                else acc = __builtin_fma((double)vi[u], (double)xv[u], acc);
            }
    }
    return acc;
}

// Two chunks of one wavefront at once (c1 only when `two`): twice the loads
// in flight of sell_row, each row summed in the same order.
template <typename V>
__device__ __forceinline__ void sell_rows2(const int64_t* __restrict__ chunk_ptr, const int32_t* __restrict__ col,
                                           const float* __restrict__ val, const V* __restrict__ v, int64_t c0,
                                           int64_t c1, bool two, int lane, float& a0, float& a1) {
    const int64_t b0 = chunk_ptr[c0];
    const int w0 = (int)((chunk_ptr[c0 + 1] - b0) / SELL_C);
    const int64_t b1 = two ? chunk_ptr[c1] : 0;
    const int w1 = two ? (int)((chunk_ptr[c1 + 1] - b1) / SELL_C) : 0;
    const int w = w0 > w1 ? w0 : w1;
    a0 = 0.0f;
    a1 = 0.0f;
    for (int j = 0; j < w; j += SELL_UNROLL) {
        int i0[SELL_UNROLL], i1[SELL_UNROLL];
        float v0[SELL_UNROLL], v1[SELL_UNROLL], x0[SELL_UNROLL], x1[SELL_UNROLL];
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) {
            i0[u] = -1;
            v0[u] = 0.0f;
            i1[u] = -1;
            v1[u] = 0.0f;
            const int64_t off = (int64_t)(j + u) * SELL_C + lane;
            if (j + u < w0) {
                i0[u] = __builtin_nontemporal_load(col + b0 + off);
                v0[u] = __builtin_nontemporal_load(val + b0 + off);
            }
            if (j + u < w1) {
                i1[u] = __builtin_nontemporal_load(col + b1 + off);
                v1[u] = __builtin_nontemporal_load(val + b1 + off);
            }
        }
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) {
            x0[u] = i0[u] >= 0 ? (float)v[i0[u]] : 0.0f;
            x1[u] = i1[u] >= 0 ? (float)v[i1[u]] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) {
            if (i0[u] >= 0) a0 = __builtin_fmaf(v0[u], x0[u], a0);
            if (i1[u] >= 0) a1 = __builtin_fmaf(v1[u], x1[u], a1);
        }
    }
}

// dinv[i] = 1 / (sum of row i's entries in column i); *bad = 1 if that sum
// is not positive for some row.
__global__ void __launch_bounds__(SELL_C * SELL_WAVES)
    k_sell_dinv(int64_t nrows, int64_t nchunks, const int64_t* __restrict__ chunk_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val, const int32_t* __restrict__ perm,
                float* __restrict__ dinv, int* bad) {
    const int64_t c = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * SELL_WAVES + (threadIdx.x >> 6);
    if (c >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const int64_t s = c * SELL_C + lane;
    if (s >= nrows) return;
    const int32_t row = perm ? perm[s] : (int32_t)s;
    const int64_t base = chunk_ptr[c];
    const int w = (int)((chunk_ptr[c + 1] - base) / SELL_C);
    float d = 0.0f;
    for (int j = 0; j < w; ++j)
        if (col[base + (int64_t)j * SELL_C + lane] == row) d += val[base + (int64_t)j * SELL_C + lane];
    if (d > 0.0f) {
        dinv[row] = 1.0f / d;
    } else {
        dinv[row] = 0.0f;
        *bad = 1;
    }
}

// Start of a segment: zero = 1: r = b, x = 0; zero = 0: r holds the restart
// residual. p = D^-1 r (the next iteration's direction buffer); partials
// {r.z, r.r}.
__global__ void __launch_bounds__(SNT) k_sell_start(int64_t n, const float* __restrict__ b, float* __restrict__ r,
                                                    double* __restrict__ x, const float* __restrict__ dinv,
                                                    float* __restrict__ p0, float* __restrict__ p1,
                                                    const SellState* __restrict__ st, double* __restrict__ part,
                                                    int zero) {
    __shared__ double scratch[32];
    float* __restrict__ p = (zero ? 1 : st->iters + 1) & 1 ? p1 : p0;
    int64_t lo, hi;
    unsigned bl;
    block_range(n, lo, hi, bl);
    double v[2] = {0.0, 0.0};
#pragma unroll 4
    for (int64_t i = lo + threadIdx.x; i < hi; i += SNT) {
        float ri;
        if (zero) {
            ri = b[i];
            r[i] = ri;
            x[i] = 0.0;
        } else {
            ri = r[i];
        }
        const float z = dinv[i] * ri;
        p[i] = z;
        v[0] += (double)ri * (double)z;
        v[1] += (double)ri * (double)ri;
    }
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        part[2 * bl] = v[0];
        part[2 * bl + 1] = v[1];
    }
}

// q = A p and partials {p.q, 0}; also, with R64, r = fl32(b - A x) computed
// in FP64 with partials {||b - A x||^2, 0} (the true residual).
template <bool PERM, bool R64>
__global__ void __launch_bounds__(SELL_C * SELL_WAVES)
    k_sell_q(int64_t nrows, int64_t nchunks, const int64_t* __restrict__ chunk_ptr, const int32_t* __restrict__ col,
             const float* __restrict__ val, const int32_t* __restrict__ perm, const float* __restrict__ p0,
             const float* __restrict__ p1, float* __restrict__ q, const float* __restrict__ b,
             const double* __restrict__ x, double* __restrict__ part, const SellState* __restrict__ st) {
    __shared__ double scratch[32];
    if (!R64 && st->done) return;
    const float* __restrict__ p = (st->iters + 1) & 1 ? p1 : p0;
    int64_t lo, hi;
    unsigned bl;
    block_range(nchunks, lo, hi, bl);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v[2] = {0.0, 0.0};
    if (!R64) {
        for (int64_t c = lo + wv; c < hi; c += 2 * SELL_WAVES) {
            const int64_t c1 = c + SELL_WAVES;
            const bool two = c1 < hi;
            float a0, a1;
            sell_rows2<float>(chunk_ptr, col, val, p, c, c1, two, lane, a0, a1);
            const int64_t s0 = c * SELL_C + lane, s1 = c1 * SELL_C + lane;
            if (s0 < nrows) {
                const int64_t dst = PERM ? (int64_t)perm[s0] : s0;
                q[dst] = a0;
                v[0] += (double)p[dst] * (double)a0;
            }
            if (two && s1 < nrows) {
                const int64_t dst = PERM ? (int64_t)perm[s1] : s1;
                q[dst] = a1;
                v[0] += (double)p[dst] * (double)a1;
            }
        }
    }
    for (int64_t c = lo + wv; R64 && c < hi; c += SELL_WAVES) {
        const int64_t s = c * SELL_C + lane;
        if (R64) {
            const double ax = sell_row<double, double>(chunk_ptr, col, val, x, c, lane);
            if (s < nrows) {
                const int64_t dst = PERM ? (int64_t)perm[s] : s;
                const double rv = (double)b[dst] - ax;
                q[dst] = (float)rv;
                v[0] += rv * rv;
            }
        } else {
            const float ap = sell_row<float, float>(chunk_ptr, col, val, p, c, lane);
            if (s < nrows) {
                const int64_t dst = PERM ? (int64_t)perm[s] : s;
                q[dst] = ap;
                v[0] += (double)p[dst] * (double)ap;
            }
        }
    }
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        part[2 * bl] = v[0];
        part[2 * bl + 1] = 0.0;
    }
}

// r -= alpha q; partials {r.r, r.z}. x advances every second update: one
// that finds x_owed clear leaves x (the finisher then sets it), the next
// adds alpha_prev p_prev + alpha p, the two FP64 steps one per update would
// take.
__global__ void __launch_bounds__(SNT) k_sell_update(int64_t n, const float* __restrict__ p0,
                                                     const float* __restrict__ p1, const float* __restrict__ q,
                                                     float* __restrict__ r, double* __restrict__ x,
                                                     const float* __restrict__ dinv, double* __restrict__ part,
                                                     const SellState* __restrict__ st) {
    __shared__ double scratch[32];
    if (st->done) return;
    const double alpha = st->alpha, alpha_prev = st->alpha_prev;
    const float af = (float)alpha;
    const bool xstep = st->x_owed != 0;
    const float* __restrict__ p = st->iters & 1 ? p1 : p0;
    const float* __restrict__ pprev = st->iters & 1 ? p0 : p1;
    int64_t lo, hi;
    unsigned bl;
    block_range(n, lo, hi, bl);
    double v[2] = {0.0, 0.0};
#pragma unroll 4
    for (int64_t i = lo + threadIdx.x; i < hi; i += SNT) {
        // x is touched once per two iterations: non-temporal, leaving the
        // caches to r, p, q and D^-1, which the next kernels read again
        if (xstep) {
            const double t = __builtin_nontemporal_load(x + i) + alpha_prev * (double)pprev[i];
            __builtin_nontemporal_store(t + alpha * (double)p[i], x + i);
        }
        const float ri = __builtin_fmaf(-af, q[i], r[i]);
        r[i] = ri;
        const float z = dinv[i] * ri;
        v[0] += (double)ri * (double)ri;
        v[1] += (double)ri * (double)z;
    }
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        part[2 * bl] = v[0];
        part[2 * bl + 1] = v[1];
    }
}

// p = D^-1 r + beta p.
__global__ void __launch_bounds__(SNT) k_sell_direction(int64_t n, const float* __restrict__ r,
                                                        const float* __restrict__ dinv, float* __restrict__ p0,
                                                        float* __restrict__ p1, const SellState* __restrict__ st) {
    if (st->done) return;
    const float beta = (float)st->beta;
    const float* __restrict__ pold = st->iters & 1 ? p1 : p0;
    float* __restrict__ pnew = st->iters & 1 ? p0 : p1;
    int64_t lo, hi;
    unsigned bl;
    block_range(n, lo, hi, bl);
#pragma unroll 4
    for (int64_t i = lo + threadIdx.x; i < hi; i += SNT) pnew[i] = __builtin_fmaf(beta, pold[i], dinv[i] * r[i]);
}

// The step a stopped solve still owes x (x_owed): x += alpha p of the last
// update (its direction in buffer iters % 2).
__global__ void __launch_bounds__(SNT) k_sell_settle(int64_t n, double* __restrict__ x, const float* __restrict__ p0,
                                                     const float* __restrict__ p1, const SellState* __restrict__ st) {
    if (!st->x_owed) return;
    const double alpha = st->alpha;
    const float* __restrict__ p = st->iters & 1 ? p1 : p0;
    int64_t lo, hi;
    unsigned bl;
    block_range(n, lo, hi, bl);
    for (int64_t i = lo + threadIdx.x; i < hi; i += SNT) x[i] = x[i] + alpha * (double)p[i];
}

// One work-group: sums nparts partial pairs in index order and advances the
// state (see the FIN_* modes).
template <int MODE, int NT>
__global__ void __launch_bounds__(NT) k_sell_finish(const double* __restrict__ part, unsigned nparts, SellState* st,
                                                     int zero, double rtol, int maxit) {
    __shared__ double scratch[32];
    if ((MODE == FIN_ALPHA || MODE == FIN_BETA) && st->done) return;
    double v[2] = {0.0, 0.0};
    for (unsigned i = threadIdx.x; i < nparts; i += NT) {
        v[0] += part[2 * i];
        v[1] += part[2 * i + 1];
    }
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x != 0) return;
    SellState s = *st;
    if (MODE == FIN_START) {
        s.rho = v[0];
        s.rr = v[1];
        s.x_owed = 0;  // x is complete at a segment start
        if (zero) {
            s.bb = v[1];
            s.tol2 = rtol * rtol * v[1];
            s.iters = 0;
            s.maxit = maxit;
        }
        s.done = !__builtin_isfinite(v[1]) ? 2 : (s.bb == 0.0 || v[1] <= s.tol2) ? 1 : 0;
    } else if (MODE == FIN_ALPHA) {
        s.sigma = v[0];
        if (!(v[0] > 0.0) || !__builtin_isfinite(v[0])) {
            s.done = 2;
        } else {
            s.alpha_prev = s.alpha;
            s.alpha = s.rho / v[0];
            s.iters += 1;
        }
    } else if (MODE == FIN_BETA) {
        s.x_owed ^= 1;  // the update ran: it left x or added the owed step and its own
        s.rr = v[0];
        if (!__builtin_isfinite(v[0])) {
            s.done = 2;
        } else if (v[0] <= s.tol2) {
            s.done = 1;
        } else if (s.iters >= s.maxit) {
            s.done = 3;
        } else {
            s.beta = v[1] / s.rho;
            s.rho = v[1];
        }
    } else {
        s.true_rr = v[0];
    }
    *st = s;
}

// One finisher launch: 1024 threads for more than 4096 partial pairs, else
// 256 (a smaller work-group starts sooner).
template <int MODE>
void launch_finish(hipStream_t s, const double* part, unsigned nparts, SellState* st, int zero, double rtol,
                   int maxit) {
    if (nparts > 4096)
        hipLaunchKernelGGL((k_sell_finish<MODE, FNT>), dim3(1), dim3(FNT), 0, s, part, nparts, st, zero, rtol, maxit);
    else
        hipLaunchKernelGGL((k_sell_finish<MODE, SNT>), dim3(1), dim3(SNT), 0, s, part, nparts, st, zero, rtol, maxit);
}

unsigned stream_grid(int64_t n) {
    const int64_t g = (n + SNT * 4 - 1) / (SNT * 4);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, SELL_MAX_GRID));
}

unsigned chunk_grid(int64_t nchunks) {
    const int64_t g = (nchunks + SELL_WAVES - 1) / SELL_WAVES;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, SELL_MAX_QGRID));
}

}  // namespace

extern "C" {

pcg_status pcg_sell_build(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                          const float* values, int chunk, int sigma, int64_t* nchunks, int64_t* nslots,
                          int64_t* chunk_ptr, int32_t* perm, int32_t* col_out, float* val_out) {
    const int64_t IMAX = 2147483647;
    if (nrows < 0 || nrows > IMAX || ncols < 0 || ncols > IMAX)
        return serr(PCG_E_ARG, "pcg_sell_build: nrows and ncols must be in [0, 2^31 - 1]");
    if (chunk < 1 || sigma < 1 || (sigma > 1 && sigma % chunk != 0))
        return serr(PCG_E_ARG, "pcg_sell_build: chunk >= 1 and sigma = 1 or a multiple of chunk (got %d, %d)",
                    chunk, sigma);
    if (!nchunks || !nslots) return serr(PCG_E_ARG, "pcg_sell_build: null nchunks or nslots");
    if (!rowptr || (nrows > 0 && rowptr[nrows] > 0 && (!colidx || !values)))
        return serr(PCG_E_ARG, "pcg_sell_build: null compressed-row array");
    if (rowptr[0] != 0) return serr(PCG_E_ARG, "pcg_sell_build: rowptr[0] must be 0");
    for (int64_t i = 0; i < nrows; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return serr(PCG_E_ARG, "pcg_sell_build: rowptr decreases at row %lld", (long long)i);
    const int64_t nnz = rowptr[nrows];
    for (int64_t k = 0; k < nnz; ++k)
        if (colidx[k] < 0 || colidx[k] >= ncols)
            return serr(PCG_E_ARG, "pcg_sell_build: column %d of entry %lld out of range", colidx[k], (long long)k);

    // Sorted order: decreasing length inside each window of sigma rows.
    std::vector<int32_t> order((size_t)nrows);
    std::iota(order.begin(), order.end(), 0);
    if (sigma > 1)
        for (int64_t w0 = 0; w0 < nrows; w0 += sigma) {
            const int64_t w1 = std::min<int64_t>(w0 + sigma, nrows);
            std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int32_t a, int32_t b) {
                return rowptr[a + 1] - rowptr[a] > rowptr[b + 1] - rowptr[b];
            });
        }
    const int64_t nch = (nrows + chunk - 1) / chunk;
    int64_t slots = 0;
    std::vector<int64_t> cptr((size_t)nch + 1);
    for (int64_t c = 0; c < nch; ++c) {
        cptr[c] = slots;
        int64_t w = 0;
        for (int64_t s = c * chunk; s < std::min<int64_t>((c + 1) * chunk, nrows); ++s) {
            const int32_t r = order[s];
            w = std::max<int64_t>(w, rowptr[r + 1] - rowptr[r]);
        }
        slots += w * chunk;
    }
    cptr[nch] = slots;
    *nchunks = nch;
    *nslots = slots;
    if (!chunk_ptr && !perm && !col_out && !val_out) return PCG_OK;
    if (!chunk_ptr || (nrows > 0 && !perm) || (slots > 0 && (!col_out || !val_out)))
        return serr(PCG_E_ARG, "pcg_sell_build: output arrays must all be given");
    std::memcpy(chunk_ptr, cptr.data(), sizeof(int64_t) * (size_t)(nch + 1));
    if (nrows) std::memcpy(perm, order.data(), sizeof(int32_t) * (size_t)nrows);
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t w = (cptr[c + 1] - cptr[c]) / chunk;
        for (int64_t l = 0; l < chunk; ++l) {
            const int64_t s = c * chunk + l;
            const int64_t len = s < nrows ? rowptr[order[s] + 1] - rowptr[order[s]] : 0;
            const int64_t k0 = s < nrows ? rowptr[order[s]] : 0;
            for (int64_t j = 0; j < w; ++j) {
                const int64_t slot = cptr[c] + j * chunk + l;
                col_out[slot] = j < len ? colidx[k0 + j] : -1;
                val_out[slot] = j < len ? values[k0 + j] : 0.0f;
            }
        }
    }
    return PCG_OK;
}

pcg_status pcg_sell_destroy(pcg_sell A) {
    if (!A) return PCG_OK;
    (void)hipFree(A->chunk_ptr);
    (void)hipFree(A->col);
    (void)hipFree(A->val);
    (void)hipFree(A->perm);
    (void)hipFree(A->r);
    (void)hipFree(A->p);
    (void)hipFree(A->p2);
    (void)hipFree(A->q);
    (void)hipFree(A->dinv);
    (void)hipFree(A->part);
    (void)hipFree(A->st);
    (void)hipFree(A->bad);
    if (A->batch) (void)hipGraphExecDestroy(A->batch);
    if (A->capture) (void)hipStreamDestroy(A->capture);
    delete A;
    return PCG_OK;
}

pcg_status pcg_sell_create(pcg_sell* out, int64_t nrows, int64_t ncols, const int64_t* rowptr,
                           const int32_t* colidx, const float* values, int sigma, void* hip_stream) {
    if (!out) return serr(PCG_E_ARG, "pcg_sell_create: null output handle");
    *out = nullptr;
    int64_t nch = 0, slots = 0;
    pcg_status st = pcg_sell_build(nrows, ncols, rowptr, colidx, values, SELL_C, sigma, &nch, &slots, nullptr,
                                   nullptr, nullptr, nullptr);
    if (st != PCG_OK) return st;
    std::vector<int64_t> cptr((size_t)nch + 1);
    std::vector<int32_t> perm((size_t)nrows), col((size_t)slots);
    std::vector<float> val((size_t)slots);
    st = pcg_sell_build(nrows, ncols, rowptr, colidx, values, SELL_C, sigma, &nch, &slots, cptr.data(),
                        perm.data(), col.data(), val.data());
    if (st != PCG_OK) return st;
    auto* A = new (std::nothrow) pcg_sell_s;
    if (!A) return serr(PCG_E_NOMEM, "pcg_sell_create: out of host memory");
    A->nrows = nrows;
    A->ncols = ncols;
    A->nnz = rowptr[nrows];
    A->nchunks = nch;
    A->nslots = slots;
    A->stream = (hipStream_t)hip_stream;
    auto alloc = [&](void** p, size_t bytes) -> hipError_t { return bytes ? hipMalloc(p, bytes) : hipSuccess; };
    hipError_t e = alloc((void**)&A->chunk_ptr, sizeof(int64_t) * (size_t)(nch + 1));
    if (e == hipSuccess) e = alloc((void**)&A->col, sizeof(int32_t) * (size_t)slots);
    if (e == hipSuccess) e = alloc((void**)&A->val, sizeof(float) * (size_t)slots);
    if (e == hipSuccess && sigma > 1) e = alloc((void**)&A->perm, sizeof(int32_t) * (size_t)nrows);
    if (e == hipSuccess)
        e = hipMemcpy(A->chunk_ptr, cptr.data(), sizeof(int64_t) * (size_t)(nch + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && slots) e = hipMemcpy(A->col, col.data(), sizeof(int32_t) * (size_t)slots, hipMemcpyHostToDevice);
    if (e == hipSuccess && slots) e = hipMemcpy(A->val, val.data(), sizeof(float) * (size_t)slots, hipMemcpyHostToDevice);
    if (e == hipSuccess && A->perm)
        e = hipMemcpy(A->perm, perm.data(), sizeof(int32_t) * (size_t)nrows, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pcg_sell_destroy(A);
        return serr(e == hipErrorOutOfMemory ? PCG_E_NOMEM : PCG_E_HIP, "pcg_sell_create: %s", hipGetErrorString(e));
    }
    *out = A;
    return PCG_OK;
}

pcg_status pcg_sell_info(pcg_sell A, int64_t* nnz, int64_t* nslots, int64_t* nchunks) {
    if (!A) return serr(PCG_E_ARG, "pcg_sell_info: null handle");
    if (nnz) *nnz = A->nnz;
    if (nslots) *nslots = A->nslots;
    if (nchunks) *nchunks = A->nchunks;
    return PCG_OK;
}

pcg_status pcg_sell_spmv(pcg_sell A, const float* x, float* y) {
    if (!A) return serr(PCG_E_ARG, "pcg_sell_spmv: null handle");
    if (A->nrows == 0) return PCG_OK;
    if (!y || (A->ncols > 0 && !x)) return serr(PCG_E_ARG, "pcg_sell_spmv: null pointer");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 3u)
        return serr(PCG_E_ARG, "pcg_sell_spmv: x and y must be 4-byte aligned");
    const auto xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    const uintptr_t xb = (uintptr_t)A->ncols * 4, yb = (uintptr_t)A->nrows * 4;
    if (xb > 0 && xa < ya + yb && ya < xa + xb) return serr(PCG_E_ARG, "pcg_sell_spmv: x and y overlap");
    const int64_t blocks = (A->nchunks + SELL_WAVES - 1) / SELL_WAVES;
    const dim3 grid((unsigned)blocks), block(SELL_C * SELL_WAVES);
    if (A->perm)
        hipLaunchKernelGGL(k_sell_spmv<true>, grid, block, 0, A->stream, A->nrows, A->nchunks, A->chunk_ptr, A->col,
                           A->val, A->perm, x, y);
    else
        hipLaunchKernelGGL(k_sell_spmv<false>, grid, block, 0, A->stream, A->nrows, A->nchunks, A->chunk_ptr, A->col,
                           A->val, A->perm, x, y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return serr(PCG_E_HIP, "pcg_sell_spmv: launch failed: %s", hipGetErrorString(e));
    return PCG_OK;
}

// Workspace and Jacobi diagonal of the solver (first call only).
static pcg_status sell_prepare(pcg_sell A) {
    if (A->diag_state == 0) {
        const size_t n = (size_t)A->nrows;
        const size_t nparts = 2 * (size_t)std::max(stream_grid(A->nrows), chunk_grid(A->nchunks));
        hipError_t e = hipMalloc((void**)&A->r, n * 4);
        if (e == hipSuccess) e = hipMalloc((void**)&A->p, n * 4);
        if (e == hipSuccess) e = hipMalloc((void**)&A->p2, n * 4);
        if (e == hipSuccess) e = hipMalloc((void**)&A->q, n * 4);
        if (e == hipSuccess) e = hipMalloc((void**)&A->dinv, n * 4);
        if (e == hipSuccess) e = hipMalloc((void**)&A->part, nparts * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void**)&A->st, sizeof(SellState));
        if (e == hipSuccess) e = hipMalloc((void**)&A->bad, sizeof(int));
        if (e == hipSuccess) e = hipMemsetAsync(A->bad, 0, sizeof(int), A->stream);
        if (e == hipSuccess) e = hipMemsetAsync(A->st, 0, sizeof(SellState), A->stream);
        if (e == hipSuccess) {
            const dim3 grid((unsigned)((A->nchunks + SELL_WAVES - 1) / SELL_WAVES)), block(SELL_C * SELL_WAVES);
            hipLaunchKernelGGL(k_sell_dinv, grid, block, 0, A->stream, A->nrows, A->nchunks, A->chunk_ptr, A->col,
                               A->val, A->perm, A->dinv, A->bad);
            e = hipGetLastError();
        }
        int bad = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, A->bad, sizeof(int), hipMemcpyDeviceToHost, A->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(A->stream);
        if (e != hipSuccess)
            return serr(e == hipErrorOutOfMemory ? PCG_E_NOMEM : PCG_E_HIP, "pcg_sell_solve: %s", hipGetErrorString(e));
        A->diag_state = bad ? -1 : 1;
    }
    if (A->diag_state < 0)
        return serr(PCG_E_ARG, "pcg_sell_solve: the matrix has a row whose diagonal is missing or not positive");
    return PCG_OK;
}

pcg_status pcg_sell_solve(pcg_sell A, const float* b, double* x, double rtol, int maxit, pcg_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!A) return serr(PCG_E_ARG, "pcg_sell_solve: null handle");
    if (A->nrows != A->ncols) return serr(PCG_E_ARG, "pcg_sell_solve: the matrix must be square");
    if (!(rtol >= 0.0) || maxit < 0) return serr(PCG_E_ARG, "pcg_sell_solve: rtol must be >= 0 and maxit >= 0");
    pcg_info out{};
    const int64_t n = A->nrows;
    if (n == 0) {
        if (info) *info = out;
        return PCG_OK;
    }
    if (!b || !x) return serr(PCG_E_ARG, "pcg_sell_solve: null pointer");
    if ((reinterpret_cast<uintptr_t>(b) & 3u) || (reinterpret_cast<uintptr_t>(x) & 7u))
        return serr(PCG_E_ARG, "pcg_sell_solve: b must be 4-byte and x 8-byte aligned");
    {
        const auto ba = reinterpret_cast<uintptr_t>(b), xa = reinterpret_cast<uintptr_t>(x);
        if (ba < xa + (uintptr_t)n * 8 && xa < ba + (uintptr_t)n * 4)
            return serr(PCG_E_ARG, "pcg_sell_solve: b and x overlap");
    }
    pcg_status ps = sell_prepare(A);
    if (ps != PCG_OK) return ps;

    hipStream_t s = A->stream;
    const unsigned gs = stream_grid(n), gq = chunk_grid(A->nchunks);
    const dim3 bs(SNT), bq(SELL_C * SELL_WAVES);
    auto q_kernel = [&](bool r64, hipStream_t qs) {
        const float* pp = A->p;
        const float* pp2 = A->p2;
        if (A->perm) {
            if (r64) hipLaunchKernelGGL((k_sell_q<true, true>), dim3(gq), bq, 0, qs, n, A->nchunks, A->chunk_ptr, A->col, A->val, A->perm, pp, pp2, A->r, b, x, A->part, A->st);
            else hipLaunchKernelGGL((k_sell_q<true, false>), dim3(gq), bq, 0, qs, n, A->nchunks, A->chunk_ptr, A->col, A->val, A->perm, pp, pp2, A->q, b, x, A->part, A->st);
        } else {
            if (r64) hipLaunchKernelGGL((k_sell_q<false, true>), dim3(gq), bq, 0, qs, n, A->nchunks, A->chunk_ptr, A->col, A->val, A->perm, pp, pp2, A->r, b, x, A->part, A->st);
            else hipLaunchKernelGGL((k_sell_q<false, false>), dim3(gq), bq, 0, qs, n, A->nchunks, A->chunk_ptr, A->col, A->val, A->perm, pp, pp2, A->q, b, x, A->part, A->st);
        }
    };
    SellState hs{};
    auto read_state = [&]() -> hipError_t {
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&hs, A->st, sizeof(SellState), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
#define SCHK(expr)                                                                                         \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return serr(PCG_E_HIP, "pcg_sell_solve: %s", hipGetErrorString(e_));     \
    } while (0)
    constexpr int BATCH = 16;  // iterations enqueued between state reads
    // k iterations on stream es (rtol and maxit are not read by these
    // finishers: the state holds them, so a captured batch does not depend on them)
    auto enqueue = [&](int k, hipStream_t es) -> hipError_t {
        for (int it = 0; it < k; ++it) {
            q_kernel(false, es);
            launch_finish<FIN_ALPHA>(es, A->part, gq, A->st, 0, 0.0, 0);
            hipLaunchKernelGGL(k_sell_update, dim3(gs), bs, 0, es, n, A->p, A->p2, A->q, A->r, x, A->dinv, A->part,
                               A->st);
            launch_finish<FIN_BETA>(es, A->part, gs, A->st, 0, 0.0, 0);
            hipLaunchKernelGGL(k_sell_direction, dim3(gs), bs, 0, es, n, A->r, A->dinv, A->p, A->p2, A->st);
        }
        return hipGetLastError();
    };
    auto ensure_batch = [&](const double* xp) -> hipError_t {
        if (A->batch && A->batch_x == xp) return hipSuccess;
        if (A->batch) {
            (void)hipGraphExecDestroy(A->batch);
            A->batch = nullptr;
        }
        hipError_t e = hipSuccess;
        if (!A->capture) e = hipStreamCreateWithFlags(&A->capture, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipStreamBeginCapture(A->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipError_t ek = enqueue(BATCH, A->capture);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(A->capture, &g);
        if (ek != hipSuccess || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return ek != hipSuccess ? ek : ec;
        }
        e = hipGraphInstantiate(&A->batch, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            A->batch = nullptr;
            return e;
        }
        A->batch_x = xp;
        return hipSuccess;
    };
    int restarts = 0;
    double rel_true = 0.0;
    for (int zero = 1;; zero = 0) {
        hipLaunchKernelGGL(k_sell_start, dim3(gs), bs, 0, s, n, b, A->r, x, A->dinv, A->p, A->p2, A->st, A->part,
                           zero);
        launch_finish<FIN_START>(s, A->part, gs, A->st, zero, rtol, maxit);
        SCHK(read_state());
        while (!hs.done && hs.iters < maxit) {
            const int k = std::min(BATCH, maxit - hs.iters);
            if (k == BATCH && A->use_graph) {
                SCHK(ensure_batch(x));
                SCHK(hipGraphLaunch(A->batch, s));
            } else {
                SCHK(enqueue(k, s));
            }
            SCHK(read_state());
        }
        // x takes the step it still owes, then the FP64 true residual; r =
        // fl32(b - A x) is the restart residual.
        hipLaunchKernelGGL(k_sell_settle, dim3(gs), bs, 0, s, n, x, A->p, A->p2, A->st);
        q_kernel(true, s);
        launch_finish<FIN_TRUE>(s, A->part, gq, A->st, 0, rtol, maxit);
        SCHK(read_state());
        rel_true = hs.bb > 0.0 ? std::sqrt(hs.true_rr / hs.bb) : 0.0;
        if (hs.done == 1 && rel_true > rtol && restarts < A->max_restarts && hs.iters < maxit) {
            ++restarts;
            continue;
        }
        break;
    }
#undef SCHK
    const pcg_status status = hs.done == 1 ? (rel_true <= rtol ? PCG_OK : PCG_E_TRUE_RESIDUAL)
                              : hs.done == 2 ? PCG_E_BREAKDOWN : PCG_E_NOCONV;
    out.iters = hs.iters;
    out.status = status;
    out.rel_res_recursive = hs.bb > 0.0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
    out.rel_res_true_fp64 = rel_true;
    out.restarts = restarts;
    out.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = out;
    if (status == PCG_E_BREAKDOWN) serr(status, "pcg_sell_solve: breakdown (p.Ap <= 0 or a non-finite value)");
    if (status == PCG_E_NOCONV) serr(status, "pcg_sell_solve: %d iterations without convergence", hs.iters);
    if (status == PCG_E_TRUE_RESIDUAL)
        serr(status, "pcg_sell_solve: the FP64 true residual %.3e is above rtol %.3e after %d restarts", rel_true, rtol,
             restarts);
    return status;
}

pcg_status pcg_sell_set_graph(pcg_sell A, int use_graph) {
    if (!A) return serr(PCG_E_ARG, "pcg_sell_set_graph: null handle");
    A->use_graph = use_graph ? 1 : 0;
    return PCG_OK;
}

pcg_status pcg_sell_set_restarts(pcg_sell A, int max_restarts) {
    if (!A) return serr(PCG_E_ARG, "pcg_sell_set_restarts: null handle");
    if (max_restarts < -1) return serr(PCG_E_ARG, "pcg_sell_set_restarts: max_restarts must be >= -1");
    A->max_restarts = max_restarts < 0 ? 3 : max_restarts;
    return PCG_OK;
}

}  // extern "C"
