// ops.hpp -- loaders, per-point operations and grid-reduction finishers that
// turn the z-march skeleton into the stencil apply, the two fused PCG
// iteration kernels and the FP64 true-residual kernel.
#pragma once

#include "zmarch.hpp"

namespace pcgmi {

// Device-resident scalars of one solve. Written by one work-group of a
// kernel (the last to finish a grid reduction, work-group 0 of a chained PCG
// kernel into the other of the two state buffers, or the init kernel) and
// read by later kernels, so kernel boundaries order every access.
struct SolveState {
    double rho;    // r.z of the current residual
    double alpha;  // rho / (p.Ap) of the current iteration
    double beta;   // rho_new / rho_old for the next direction
    double sigma;  // p.Ap
    double rr;     // ||r||^2 of the current residual
    double rr0;    // ||b||^2
    double tol2;   // (rtol ||b||)^2
    double dinv;   // 1 / diagonal (constant-coefficient operator)
    int iters;     // completed iterations
    int done;      // 0 running, 1 converged, 2 breakdown, 3 maxit reached, 4 stagnated
    int maxit;
    int stag;      // > 0: stop when the best ||r|| has not improved by 10% for stag iterations
    int stag_at;   // iteration of the last 10% improvement of the best residual
    double stag_best;  // best relative residual at that iteration
    // flexible CG
    int flags;        // FLEX_JACOBI: preconditioner is D^-1; FLEX_RESTART: next beta = 0; FLEX_REDO
    int fallback_at;  // iteration of the switch to Jacobi (-1: none)
    double zr;        // z.r of the last preconditioned residual
    double alpha_prev;  // alpha of the iteration before (x advanced every second iteration)
};
// FLEX_MG: the preconditioned residual z is the multigrid V-cycle's, taken as it is.
constexpr int FLEX_JACOBI = 1, FLEX_RESTART = 2, FLEX_REDO = 4, FLEX_MG = 8;
// Flexible CG falls back to Jacobi when the best residual has not improved
// by 10% for this many iterations. CG plateaus on the 128^3
// variable-coefficient operator outlast 20 iterations even with plain
// Jacobi (measured), so the window is the one refinement's inner stop uses.
constexpr int FLEX_STAG_WINDOW = 100;

// ---------------------------------------------------------------- loaders
// A loader provides Raw<N> (registers of one fetch of N consecutive points),
// fetch<N>(idx, raw) (issue the loads) and finish<N>(raw, out) (compute-type
// values of the field at those points).

// Plain load of a stored field of type T.
template <typename T> struct LoadField {
    using C = typename Traits<T>::C;
    template <int N> using Raw = RawN<T, N>;
    const T* __restrict__ x;
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const { r.load(x + i); }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = r.get(v);
    }
};

// Load of a field of type S widened to the compute type C (e.g. an FP32
// iterate read by an FP64 kernel).
template <typename S, typename C> struct LoadWiden {
    template <int N> using Raw = RawN<S, N>;
    const S* __restrict__ x;
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const { r.load(x + i); }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = (C)r.get(v);
    }
};

// New search direction computed on the fly: p = stored(dinv * r + beta * p_old).
// beta comes from the solve state; dinv is the constant Jacobi scale.
template <typename T> struct LoadDirection {
    using C = typename Traits<T>::C;
    template <int N> struct Raw {
        RawN<T, N> r, p;
    };
    const T* __restrict__ r;
    const T* __restrict__ pold;
    const SolveState* st;
    C beta, dinv;
    __device__ void init() {
        beta = (C)st->beta;
        dinv = (C)st->dinv;
    }
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& raw) const {
        raw.r.load(r + i);
        raw.p.load(pold + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& raw, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = stored<T>(dinv * raw.r.get(v) + beta * raw.p.get(v));
    }
};

// Variable coefficients: the field x (type T) together with the cell
// coefficient k (FP32) of each point.
template <typename T> struct LoadUK {
    using C = typename Traits<T>::C;
    template <int N> struct Raw {
        RawN<T, N> u;
        RawN<float, N> k;
    };
    const T* __restrict__ x;
    const float* __restrict__ kc;
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const {
        r.u.load(x + i);
        r.k.load(kc + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, UK<C>* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = UK<C>{r.u.get(v), (C)r.k.get(v)};
    }
};

// Field of type S widened to C, with k (variable-coefficient FP64 kernels).
template <typename S, typename C> struct LoadWidenUK {
    template <int N> struct Raw {
        RawN<S, N> u;
        RawN<float, N> k;
    };
    const S* __restrict__ x;
    const float* __restrict__ kc;
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const {
        r.u.load(x + i);
        r.k.load(kc + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, UK<C>* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = UK<C>{(C)r.u.get(v), (C)r.k.get(v)};
    }
};

// The cell coefficient alone (for the diagonal of the variable operator).
template <typename C> struct LoadK {
    template <int N> using Raw = RawN<float, N>;
    const float* __restrict__ kc;
    __device__ void init() {}
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& r) const { r.load(kc + i); }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& r, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = (C)r.get(v);
    }
};

// Direction with a variable Jacobi scale: p = stored(dinv_p r + beta p_old), with k.
template <typename T> struct LoadDirectionVar {
    using C = typename Traits<T>::C;
    template <int N> struct Raw {
        RawN<T, N> r, p, d;
        RawN<float, N> k;
    };
    const T* __restrict__ r;
    const T* __restrict__ pold;
    const T* __restrict__ dinv;
    const float* __restrict__ kc;
    const SolveState* st;
    C beta;
    __device__ void init() { beta = (C)st->beta; }
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& raw) const {
        raw.r.load(r + i);
        raw.p.load(pold + i);
        raw.d.load(dinv + i);
        raw.k.load(kc + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& raw, UK<C>* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v)
            out[v] = UK<C>{stored<T>(raw.d.get(v) * raw.r.get(v) + beta * raw.p.get(v)), (C)raw.k.get(v)};
    }
};

// Single-reduction PCG (Chronopoulos-Gear): the preconditioned new
// residual u_{i+1} = D^-1 r_{i+1}, with s_i = stored(w_i + beta s_{i-1}) and
// r_{i+1} = stored(r_i - alpha s_i) computed on the fly for the tile and its
// halo (constant Jacobi scale).
template <typename T> struct LoadSR {
    using C = typename Traits<T>::C;
    template <int N> struct Raw {
        RawN<T, N> r, w, s;
    };
    const T* __restrict__ r;
    const T* __restrict__ w;
    const T* __restrict__ s;
    const SolveState* st;
    C alpha, beta, dinv;
    __device__ void init() {
        alpha = (C)st->alpha;
        beta = (C)st->beta;
        dinv = (C)st->dinv;
    }
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& raw) const {
        raw.r.load(r + i);
        raw.w.load(w + i);
        raw.s.load(s + i);
    }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& raw, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) {
            const C sv = stored<T>(raw.w.get(v) + beta * raw.s.get(v));
            out[v] = dinv * stored<T>(raw.r.get(v) - alpha * sv);
        }
    }
};

// u = D^-1 r (constant Jacobi scale), not rounded: the start of the
// single-reduction form.
template <typename T> struct LoadPrecond {
    using C = typename Traits<T>::C;
    template <int N> using Raw = RawN<T, N>;
    const T* __restrict__ r;
    const SolveState* st;
    C dinv;
    __device__ void init() { dinv = (C)st->dinv; }
    template <int N> __device__ __forceinline__ void fetch(int64_t i, Raw<N>& raw) const { raw.load(r + i); }
    template <int N> __device__ __forceinline__ void finish(const Raw<N>& raw, C* out) const {
#pragma unroll
        for (int v = 0; v < N; ++v) out[v] = dinv * raw.get(v);
    }
};

// ---------------------------------------------------------------- store helpers

template <typename T, int VX>
__device__ __forceinline__ void st_pts(T* __restrict__ p, int64_t i, const typename Traits<T>::C* in) {
    if constexpr (VX == Traits<T>::W) store_vec<T>(p + i, in);
    else {
#pragma unroll
        for (int v = 0; v < VX; ++v) p[i + v] = from_c<T>(in[v]);
    }
}

// Non-temporal form of st_pts, for outputs no later kernel of the solve
// re-reads soon (they bypass L2 and the last-level cache).
template <typename T, int VX>
__device__ __forceinline__ void st_pts_nt(T* __restrict__ p, int64_t i, const typename Traits<T>::C* in) {
    if constexpr (VX == Traits<T>::W) store_vec_nt<T>(p + i, in);
    else {
#pragma unroll
        for (int v = 0; v < VX; ++v) p[i + v] = from_c<T>(in[v]);
    }
}

// Store N values of compute type to X (a double accumulator or a storage type).
template <typename X, int N>
__device__ __forceinline__ void st_any(X* __restrict__ p, int64_t i, const double* in) {
    constexpr int W = 16 / (int)sizeof(X);
    if constexpr (N % W == 0) {
#pragma unroll
        for (int j = 0; j < N / W; ++j) {
            typename Traits<X>::C t[W];
#pragma unroll
            for (int e = 0; e < W; ++e) t[e] = (typename Traits<X>::C)in[j * W + e];
            store_vec<X>(p + i + j * W, t);
        }
    } else {
#pragma unroll
        for (int v = 0; v < N; ++v) p[i + v] = from_c<X>((typename Traits<X>::C)in[v]);
    }
}

template <typename X, int N>
__device__ __forceinline__ void st_any_nt(X* __restrict__ p, int64_t i, const double* in) {
    constexpr int W = 16 / (int)sizeof(X);
    if constexpr (N % W == 0) {
#pragma unroll
        for (int j = 0; j < N / W; ++j) {
            typename Traits<X>::C t[W];
#pragma unroll
            for (int e = 0; e < W; ++e) t[e] = (typename Traits<X>::C)in[j * W + e];
            store_vec_nt<X>(p + i + j * W, t);
        }
    } else {
#pragma unroll
        for (int v = 0; v < N; ++v) p[i + v] = from_c<X>((typename Traits<X>::C)in[v]);
    }
}

// ---------------------------------------------------------------- ops
// An op provides Raw (registers of its own streams at one thread's points of
// one plane), fetch(idx, raw) and apply(idx, raw, c, ax, acc).

struct NoRaw {};

// y = A x (a non-temporal store: measured 5.16 -> 5.37 TB/s at 512^3 FP32)
template <typename T, int VX> struct OpStore {
    using C = typename Traits<T>::C;
    using Raw = NoRaw;
    T* __restrict__ y;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t, Raw&) const {}
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw&, const Cell* c, const C* ax, C (&acc)[NC]) const {
        st_pts_nt<T, VX>(y, i, ax);
    }
};

// Iteration kernel 1: store the new direction p (already rounded to T by the
// loader) and accumulate p.Ap.
template <typename T, int VX> struct OpDirection {
    using C = typename Traits<T>::C;
    using Raw = NoRaw;
    T* __restrict__ pnew;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t, Raw&) const {}
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw&, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C u[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            u[v] = cell_u(c[v]);
            acc[0] += u[v] * ax[v];
        }
        st_pts<T, VX>(pnew, i, u);
    }
};

// Iteration kernel 2: with q = A p recomputed from p, r = stored(r - alpha q);
// accumulate r.r of the stored residual and, with a variable Jacobi scale
// (dinv != null), r.z = sum dinv r^2 as component 1. The x accumulator (XM):
//   XM = 0: x += alpha p every iteration;
//   XM = 1: x untouched (an odd iteration when x advances every second one);
//   XM = 2: x += alpha_prev p_prev + alpha p (the even iteration after it,
//           p_prev the previous direction, still in the other p buffer).
// Nothing in the recursion reads x, so it may lag one iteration: advancing it
// every second iteration takes the x stream (16 B/pt in FP64) out of every
// other update. With an FP64 accumulator XM = 2 performs exactly the two
// FP64 steps XM = 0 would, so x keeps its bits.
// NTX: x is loaded and stored non-temporally. When an iteration's vectors
// exceed the last-level cache, x (read again only one iteration later, and
// the widest stream) then leaves the cache to r and p, which the next
// kernel re-reads: measured 126 -> 119 us per iteration at 256^3.
template <typename T, typename X, int VX, bool VAR = false, bool NTX = false, int XM = 0> struct OpUpdate {
    using C = typename Traits<T>::C;
    struct Raw {
        RawN<T, VX> r;
        RawN<X, XM == 1 ? 1 : VX> x;
        RawN<T, VAR ? VX : 1> d;
        RawN<T, XM == 2 ? VX : 1> pp;
    };
    X* __restrict__ x;
    T* __restrict__ r;
    const SolveState* st;
    const T* __restrict__ dinv;
    C alpha;
    double alpha_d;
    const T* __restrict__ pprev = nullptr;  // XM = 2: the previous direction
    double alpha_prev_d = 0.0;
    __device__ void init() {
        alpha = (C)st->alpha;
        alpha_d = (double)alpha;
        if constexpr (XM == 2) alpha_prev_d = (double)(C)st->alpha_prev;
    }
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const {
        raw.r.load(r + i);
        if constexpr (XM != 1) {
            if constexpr (NTX) raw.x.load_nt(x + i);
            else raw.x.load(x + i);
        }
        if constexpr (VAR) raw.d.load(dinv + i);
        if constexpr (XM == 2) raw.pp.load(pprev + i);
    }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C rv[VX];
        double xv[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            if constexpr (XM == 0) {
                xv[v] = (double)raw.x.get(v) + alpha_d * (double)cell_u(c[v]);
            } else if constexpr (XM == 2) {
                const double t = (double)raw.x.get(v) + alpha_prev_d * (double)raw.pp.get(v);
                xv[v] = t + alpha_d * (double)cell_u(c[v]);
            }
            rv[v] = stored<T>(raw.r.get(v) - alpha * ax[v]);
            acc[0] += rv[v] * rv[v];
            if constexpr (VAR) acc[NC - 1] += raw.d.get(v) * rv[v] * rv[v];
        }
        if constexpr (XM != 1) {
            if constexpr (NTX) st_any_nt<X, VX>(x, i, xv);
            else st_any<X, VX>(x, i, xv);
        }
        st_pts<T, VX>(r, i, rv);
    }
};

// Single-reduction iteration: with u_{i+1} (the cell) and w_{i+1} = A u_{i+1}
// (ax) from the stencil, and s_i, r_{i+1} recomputed exactly as the loader
// did: p_i = stored(D^-1 r_i + beta p_{i-1}) (in place), x += alpha p_i,
// stores s_i, r_{i+1}, w_{i+1}; accumulates gamma = r.u, delta = w.u and
// ||r||^2 of the new residual.
template <typename T, typename X, int VX> struct OpSR {
    using C = typename Traits<T>::C;
    struct Raw {
        RawN<T, VX> r, w, s, p;
        RawN<X, VX> x;
    };
    const T* __restrict__ r_in;
    const T* __restrict__ w_in;
    const T* __restrict__ s_in;
    T* __restrict__ r_out;
    T* __restrict__ w_out;
    T* __restrict__ s_out;
    T* __restrict__ p;
    X* __restrict__ x;
    const SolveState* st;
    C alpha, beta, dinv;
    double alpha_d;
    __device__ void init() {
        alpha = (C)st->alpha;
        beta = (C)st->beta;
        dinv = (C)st->dinv;
        alpha_d = (double)alpha;
    }
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const {
        raw.r.load(r_in + i);
        raw.w.load(w_in + i);
        raw.s.load(s_in + i);
        raw.p.load(p + i);
        raw.x.load(x + i);
    }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C sv[VX], rn[VX], pv[VX], wn[VX];
        double xv[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            sv[v] = stored<T>(raw.w.get(v) + beta * raw.s.get(v));
            rn[v] = stored<T>(raw.r.get(v) - alpha * sv[v]);
            pv[v] = stored<T>(dinv * raw.r.get(v) + beta * raw.p.get(v));
            xv[v] = (double)raw.x.get(v) + alpha_d * (double)pv[v];
            wn[v] = stored<T>(ax[v]);
            const C un = cell_u(c[v]);
            acc[0] += rn[v] * un;
            acc[1] += wn[v] * un;
            acc[2] += rn[v] * rn[v];
        }
        st_pts<T, VX>(s_out, i, sv);
        st_pts<T, VX>(r_out, i, rn);
        st_pts<T, VX>(w_out, i, wn);
        st_pts<T, VX>(p, i, pv);
        st_any<X, VX>(x, i, xv);
    }
};

// Start of the single-reduction form: w = stored(A u) with u = D^-1 r (the
// cell); accumulates gamma = r.u and delta = w.u.
template <typename T, int VX> struct OpSRStart {
    using C = typename Traits<T>::C;
    struct Raw {
        RawN<T, VX> r;
    };
    const T* __restrict__ r;
    T* __restrict__ w;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const { raw.r.load(r + i); }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C wn[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            wn[v] = stored<T>(ax[v]);
            const C un = cell_u(c[v]);
            acc[0] += raw.r.get(v) * un;
            acc[1] += wn[v] * un;
        }
        st_pts<T, VX>(w, i, wn);
    }
};

// dinv = 1 / D with D the variable operator's diagonal (from StencilVarDiag).
template <typename T, int VX> struct OpStoreInverse {
    using C = typename Traits<T>::C;
    using Raw = NoRaw;
    T* __restrict__ dinv;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t, Raw&) const {}
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw&, const Cell* c, const C* ax, C (&acc)[NC]) const {
        C out[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) out[v] = C(1) / ax[v];
        st_pts<T, VX>(dinv, i, out);
    }
};

// FP64 true residual: r = b - A x (not stored); accumulate ||r||^2 and max |r|.
template <typename B, int VX> struct OpResidual64 {
    struct Raw {
        RawN<B, VX> b;
    };
    const B* __restrict__ b;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const { raw.b.load(b + i); }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const double* ax,
                                          double (&acc)[NC]) const {
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            double rv = (double)raw.b.get(v) - ax[v];
            acc[0] += rv * rv;
            double a = fabs(rv);
            acc[1] = a > acc[1] ? a : acc[1];
        }
    }
};

// Scaled residual for refinement: rhat = stored(s (b - A x)) with b, x and
// the arithmetic in FP64, rounded FP64 -> FP32 -> storage type.
template <typename T, int VX> struct OpCastScaled {
    struct Raw {
        RawN<double, VX> b;
    };
    const double* __restrict__ b;
    T* __restrict__ rhat;
    double scale;
    __device__ void init() {}
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const { raw.b.load(b + i); }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const double* ax,
                                          double (&acc)[NC]) const {
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const double rv = scale * (raw.b.get(v) - ax[v]);
            rhat[i + v] = from_c<T>((typename Traits<T>::C)rv);
        }
    }
};

// Residual of an initial guess, computed in FP64 and rounded to the storage
// type (through FP32 for 16-bit types): r = stored(b - A x0); accumulates
// r.r of the stored residual, b.b and r.z = sum dinv r^2 (dinv from the array
// when given, else the constant of the solve state).
template <typename T, int VX> struct OpInitResidual {
    struct Raw {
        RawN<T, VX> b;
    };
    const T* __restrict__ b;
    T* __restrict__ r;
    const T* __restrict__ dinv;
    const SolveState* st;
    double dconst;
    __device__ void init() { dconst = st->dinv; }
    __device__ __forceinline__ void fetch(int64_t i, Raw& raw) const { raw.b.load(b + i); }
    template <int NC, class Cell>
    __device__ __forceinline__ void apply(int64_t i, const Raw& raw, const Cell* c, const double* ax,
                                          double (&acc)[NC]) const {
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const double bv = (double)raw.b.get(v);
            const T rs = from_c<T>((typename Traits<T>::C)(bv - ax[v]));
            r[i + v] = rs;
            const double rv = (double)to_c(rs);
            const double dv = dinv ? (double)to_c(dinv[i + v]) : dconst;
            acc[0] += rv * rv;
            acc[1] += bv * bv;
            acc[2] += dv * rv * rv;
        }
    }
};

// ---------------------------------------------------------------- finishers
// Run by thread 0 of the last work-group with the FP64 grid totals.

struct FinNone {
    __device__ void operator()(const double*) const {}
};

// After p.Ap: alpha = rho / sigma, or breakdown.
struct FinAlpha {
    SolveState* st;
    __device__ void operator()(const double* tot) const {
        double sigma = tot[0];
        st->sigma = sigma;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            st->done = 2;
            return;
        }
        st->alpha_prev = st->alpha;
        st->alpha = st->rho / sigma;
    }
};

// After r.r: count the iteration, test convergence, form beta. With a
// variable Jacobi scale (var), rho_new = r.z is the second total.
struct FinBeta {
    SolveState* st;
    double* hist;  // relres per iteration (maxit + 1 entries) or null
    bool var;
    __device__ void operator()(const double* tot) const {
        double rr = tot[0];
        int it = st->iters + 1;
        st->iters = it;
        st->rr = rr;
        if (hist) hist[it] = sqrt(rr / st->rr0);
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
        if (st->stag > 0) {
            const double rel = sqrt(rr / st->rr0);
            if (rel < 0.9 * st->stag_best) {
                st->stag_best = rel;
                st->stag_at = it;
            } else if (it - st->stag_at >= st->stag) {
                st->done = 4;
                return;
            }
        }
        double rho_new = var ? tot[1] : st->dinv * rr;
        st->beta = rho_new / st->rho;
        st->rho = rho_new;
    }
};

// Single-reduction form, after the start's {gamma, delta}: alpha = gamma /
// delta, beta = 0.
struct FinSRStart {
    SolveState* st;
    __device__ void operator()(const double* tot) const {
        const double gamma = tot[0], delta = tot[1];
        st->rho = gamma;
        st->beta = 0.0;
        if (!(delta > 0.0) || !isfinite(delta) || !isfinite(gamma)) {
            st->done = 2;
            return;
        }
        st->alpha = gamma / delta;
    }
};

// Single-reduction form, after an iteration's {gamma, delta, ||r||^2}: count
// the iteration, test convergence (and stagnation, as FinBeta), then beta =
// gamma / gamma_old and alpha = gamma / (delta - beta gamma / alpha_old).
struct FinSR {
    SolveState* st;
    double* hist;
    __device__ void operator()(const double* tot) const {
        const double gamma = tot[0], delta = tot[1], rr = tot[2];
        const int it = st->iters + 1;
        st->iters = it;
        st->rr = rr;
        if (hist) hist[it] = sqrt(rr / st->rr0);
        if (!isfinite(rr) || !isfinite(gamma) || !isfinite(delta)) {
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
        if (st->stag > 0) {
            const double rel = sqrt(rr / st->rr0);
            if (rel < 0.9 * st->stag_best) {
                st->stag_best = rel;
                st->stag_at = it;
            } else if (it - st->stag_at >= st->stag) {
                st->done = 4;
                return;
            }
        }
        const double beta = gamma / st->rho;
        const double denom = delta - beta * gamma / st->alpha;
        if (!(denom > 0.0) || !isfinite(denom)) {
            st->done = 2;
            return;
        }
        st->alpha = gamma / denom;
        st->beta = beta;
        st->rho = gamma;
    }
};

// Start of a solve: tot = {r.r, b.b, r.z}.
struct FinStart {
    SolveState* st;
    double* hist;
    __device__ void operator()(const double* tot) const {
        double rr = tot[0], bb = tot[1];
        st->rr0 = bb;
        st->rr = rr;
        st->tol2 = st->tol2 * bb;  // host stores rtol^2 here before the launch
        st->iters = 0;
        st->beta = 0.0;
        st->stag_at = 0;
        st->stag_best = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        st->rho = tot[2];
        if (hist) hist[0] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        if (!isfinite(rr) || !isfinite(bb)) st->done = 2;
        else if (bb == 0.0 || rr <= st->tol2) st->done = 1;
        else st->done = 0;
    }
};

// Flexible CG (flex.hip; fused into the multigrid V-cycle's last sweep).
// After z.q and z.r: beta, or a switch to Jacobi when z is not a descent
// preconditioner (z.r <= 0) or not finite.
struct FinFlexBeta {
    SolveState* st;
    bool redo_pass;
    __device__ void operator()(const double* tot) const {
        const double zq = tot[0], zr = tot[1];
        st->zr = zr;
        if (redo_pass) st->flags &= ~FLEX_REDO;
        const bool jac = st->flags & FLEX_JACOBI;
        if (!jac && (!(zr > 0.0) || !isfinite(zr) || !isfinite(zq))) {
            st->flags |= FLEX_JACOBI | FLEX_RESTART | FLEX_REDO;
            st->fallback_at = st->iters;
            return;
        }
        st->beta = (st->flags & FLEX_RESTART) ? 0.0 : -zq / st->sigma;
    }
};

// FP64 residual norms: out[0] = ||r||^2, out[1] = max |r|.
struct FinStore2 {
    double* out;
    __device__ void operator()(const double* tot) const {
        out[0] = tot[0];
        out[1] = tot[1];
    }
};

}  // namespace pcgmi
