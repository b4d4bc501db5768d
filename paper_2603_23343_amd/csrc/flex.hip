// flex.hip -- flexible conjugate gradients with one stored direction (Notay,
// SIAM J. Sci. Comput. 22(4), 2000), for a preconditioner that changes from
// one application to the next (the learned network), with the Jacobi
// preconditioner as fallback:
//
//   q = A p; sigma = p.q; alpha = (p.r) / sigma; x += alpha p; r -= alpha q
//   z = M(r); beta = -(z.q) / sigma; p = z + beta p
//
// Kernels per iteration (all skip their work once the solve state is done):
//   direction: p = z + beta p_old on the fly for the tile and its halo,
//              q = A p stored, sigma = p.q and p.r -> alpha;
//   update:    r -= alpha q, ||r||^2 -> convergence, and the
//              stagnation test that switches to Jacobi (per-work-group
//              partials, finished by a one-work-group kernel); x advances
//              every second iteration (x += alpha_prev p_old + alpha p; the
//              solver adds a step still owed when it stops);
//   M:         the network's correction (cnn_forward, scaled by rms(r)
//              from the state) or nothing when Jacobi is selected;
//   select:    z = D^-1 r, plus the correction while the network is in use
//              (z as the multigrid V-cycle left it, for that preconditioner),
//              then z.q and z.r ->
//              beta, or a switch to Jacobi when z.r <= 0 or a value is not
//              finite (the second, "redo" launch then recomputes z with
//              D^-1 and restarts the direction recurrence).
#include "zkernel.hpp"

namespace pcgmi {

namespace {

// p = stored(z + beta p_old); beta = 0 on a restart.
template <typename T> struct LoadFlexDir {
    using C = typename Traits<T>::C;
    template <int N> struct Raw {
        RawN<T, N> z, p;
    };
    const T* __restrict__ z;
    const T* __restrict__ pold;
    const SolveState* st;
    C beta;
    __device__ void init() { beta = (st->flags & FLEX_RESTART) ? C(0) : (C)st->beta; }
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& raw) const {
        raw.z.load(z + i);
        raw.p.load(pold + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& raw, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = stored<T>(raw.z.get(v) + beta * raw.p.get(v));
    }
};

template <typename T> struct LoadFlexDirVar {
    using C = typename Traits<T>::C;
    template <int N> struct Raw {
        RawN<T, N> z, p;
        RawN<float, N> k;
    };
    const T* __restrict__ z;
    const T* __restrict__ pold;
    const float* __restrict__ kc;
    const SolveState* st;
    C beta;
    __device__ void init() { beta = (st->flags & FLEX_RESTART) ? C(0) : (C)st->beta; }
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& raw) const {
        raw.z.load(z + i);
        raw.p.load(pold + i);
        raw.k.load(kc + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& raw, UK<C>* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v)
            out[v] = UK<C>{stored<T>(raw.z.get(v) + beta * raw.p.get(v)), (C)raw.k.get(v)};
    }
};

// Stores p and q = A p; accumulates p.q and p.r.
template <typename T, int VX> struct OpFlexDir {
    using C = typename Traits<T>::C;
    struct Raw {
        RawN<T, VX> r;
    };
    T* __restrict__ pnew;
    T* __restrict__ q;
    const T* __restrict__ r;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const { raw.r.load(r + i); }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C u[VX], qv[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            u[v] = cell_u(c[v]);
            qv[v] = stored<T>(ax[v]);
            acc[0] += u[v] * qv[v];
            acc[1] += u[v] * raw.r.get(v);
        }
        st_pts<T, VX>(pnew, i, u);
        st_pts<T, VX>(q, i, qv);
    }
};

struct FinFlexAlpha {
    SolveState* st;
    __device__ void operator()(const double* tot) const {
        const double sigma = tot[0], pr = tot[1];
        st->sigma = sigma;
        st->flags &= ~FLEX_RESTART;
        if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(pr)) {
            st->done = 2;
            return;
        }
        st->alpha_prev = st->alpha;
        st->alpha = pr / sigma;
    }
};

// After ||r||^2: count, test convergence; switch to Jacobi (with a restart)
// when the best residual has not improved by 10% for `stag` iterations.
struct FinFlexRes {
    SolveState* st;
    double* hist;
    __device__ void operator()(const double* tot) const {
        const double rr = tot[0];
        const int it = st->iters + 1;
        st->iters = it;
        st->rr = rr;
        const double rel = sqrt(rr / st->rr0);
        if (hist) hist[it] = rel;
        if (!isfinite(rr)) {
            st->done = 2;
            return;
        }
        if (rr <= st->tol2) {
            st->done = 1;
            return;
        }
        if (it >= st->maxit) {
            st->done = 3;
            return;
        }
        if (rel < 0.9 * st->stag_best) {
            st->stag_best = rel;
            st->stag_at = it;
        } else if (!(st->flags & FLEX_JACOBI) && st->stag > 0 && it - st->stag_at >= st->stag) {
            st->flags |= FLEX_JACOBI | FLEX_RESTART;
            st->fallback_at = it;
            st->stag_at = it;
        }
    }
};

constexpr int NT = STREAM_THREADS;

// r = stored(r - alpha q); ||r||^2. x advances every second iteration: the
// update of an odd iteration leaves it (and reads no p), that of an even one
// adds alpha_prev p_old + alpha p, the two FP64 steps one per iteration
// would take (the state counts the iterations before this one).
template <typename T>
__global__ void __launch_bounds__(NT) k_flex_update(int64_t n, const T* __restrict__ p, const T* __restrict__ pold,
                                                    const T* __restrict__ q, T* __restrict__ r,
                                                    double* __restrict__ x, SolveState* st, double* hist, Red red) {
    if (st->done) return;
    __shared__ double scratch[16];
    using C = typename Traits<T>::C;
    const C a = (C)st->alpha;
    const double ad = (double)a, apd = (double)(C)st->alpha_prev;
    const bool xstep = ((st->iters + 1) & 1) == 0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    C acc = C(0);
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        if (xstep) {
            const double t = x[i] + apd * (double)to_c(pold[i]);
            x[i] = t + ad * (double)to_c(p[i]);
        }
        const C rv = stored<T>(to_c(r[i]) - a * to_c(q[i]));
        r[i] = from_c<T>(rv);
        acc += rv * rv;
    }
    // partial per work-group; k_flex_finish applies FinFlexRes (a kernel
    // boundary instead of an agent-scope release fence per work-group)
    double v[1] = {(double)acc};
    block_reduce<1, 0u>(v, scratch);
    if (threadIdx.x == 0) red.partials[blockIdx.x] = v[0];
}

// z = D^-1 r (+ the network's correction in z unless Jacobi is selected or
// this is the redo pass); z.q, z.r -> beta.
template <typename T>
__global__ void __launch_bounds__(NT) k_flex_select(int64_t n, T* __restrict__ z, const T* __restrict__ r,
                                                    const T* __restrict__ q, const T* __restrict__ dinv,
                                                    SolveState* st, int redo_pass, Red red) {
    if (st->done) return;
    if (redo_pass && !(st->flags & FLEX_REDO)) return;
    __shared__ double scratch[32];
    using C = typename Traits<T>::C;
    const bool jac = (st->flags & FLEX_JACOBI) != 0;
    const bool given = (st->flags & FLEX_MG) != 0;  // z is the V-cycle's output
    const C dc = (C)st->dinv;
    const int64_t stride = (int64_t)gridDim.x * NT;
    C zq = C(0), zr = C(0);
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        const C rv = to_c(r[i]);
        C zv;
        const C jv = (dinv ? to_c(dinv[i]) : dc) * rv;
        // Jacobi, the V-cycle's z, or Jacobi plus the network's correction held in z
        zv = stored<T>(jac ? jv : given ? to_c(z[i]) : jv + to_c(z[i]));
        if (jac || !given) z[i] = from_c<T>(zv);  // the V-cycle's z is already stored
        zq += zv * to_c(q[i]);
        zr += zv * rv;
    }
    double v[2] = {(double)zq, (double)zr};
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        red.partials[2 * blockIdx.x] = v[0];
        red.partials[2 * blockIdx.x + 1] = v[1];
    }
}

// One work-group: sums the partials of the kernel before it in index order
// and applies its finisher, unless that kernel skipped (done, or the redo
// pass without a redo).
template <int NC, class F>
__global__ void __launch_bounds__(NT) k_flex_finish(const double* __restrict__ partials, unsigned nblocks, F fin,
                                                    const SolveState* st, int redo_pass) {
    if (st->done) return;
    if (redo_pass && !(st->flags & FLEX_REDO)) return;
    __shared__ double lds[NC * 16];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (unsigned i = threadIdx.x; i < nblocks; i += NT)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += partials[NC * i + c];
    block_reduce<NC, 0u>(acc, lds);
    if (threadIdx.x == 0) fin(acc);
}

inline unsigned nblk(int64_t n) {
    int64_t b = (n + NT * 4 - 1) / (NT * 4);
    return (unsigned)(b < 1 ? 1 : (b > DOT_MAX_BLOCKS ? DOT_MAX_BLOCKS : b));
}

}  // namespace

hipError_t launch_flex_direction(const Plan& p, const Geometry& g, OpDesc od, const float* z, const float* pold,
                                 float* pnew, float* q, const float* r, SolveState* st, Red red, hipStream_t s) {
    using T = float;
    using C = float;
    return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
        OpFlexDir<T, VX> op{pnew, q, r};
        if (od.kc) {
            LoadFlexDirVar<T> ld{z, pold, od.kc, st, C(0)};
            return run_zmarch<ZF_FLEX_DIRECTION, C, StencilVar<C>, BX, BY, VX, 2, 0u, true>(g, ld, op, FinFlexAlpha{st},
                                                                                      red, &st->done, s);
        }
        LoadFlexDir<T> ld{z, pold, st, C(0)};
        return run_zmarch<ZF_FLEX_DIRECTION, C, StencilConst<C>, BX, BY, VX, 2, 0u, true>(g, ld, op, FinFlexAlpha{st},
                                                                                    red, &st->done, s);
    });
}

hipError_t launch_flex_update(int64_t n, const float* p, const float* pold, const float* q, float* r, double* x,
                              SolveState* st, double* hist, Red red, hipStream_t s) {
    const unsigned nb = nblk(n);
    if ((size_t)nb > red.cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flex_update<float>, dim3(nb), dim3(NT), 0, s, n, p, pold, q, r, x, st, hist, red);
    hipLaunchKernelGGL((k_flex_finish<1, FinFlexRes>), dim3(1), dim3(NT), 0, s, red.partials, nb, FinFlexRes{st, hist},
                       st, 0);
    return hipGetLastError();
}

hipError_t launch_flex_select(int64_t n, float* z, const float* r, const float* q, const float* dinv, SolveState* st,
                              bool redo_pass, Red red, hipStream_t s) {
    const unsigned nb = nblk(n);
    if ((size_t)2 * nb > red.cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flex_select<float>, dim3(nb), dim3(NT), 0, s, n, z, r, q, dinv, st, redo_pass ? 1 : 0, red);
    hipLaunchKernelGGL((k_flex_finish<2, FinFlexBeta>), dim3(1), dim3(NT), 0, s, red.partials, nb,
                       FinFlexBeta{st, redo_pass}, st, redo_pass ? 1 : 0);
    return hipGetLastError();
}

}  // namespace pcgmi
