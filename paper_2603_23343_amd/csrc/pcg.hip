// pcg.hip -- the two fused kernels of one Jacobi-PCG iteration (paper
// Sec. VII composes PCG from the stencil, the dot reduction and element-wise
// updates; here they are fused so each iteration makes two passes over HBM):
//
//   kernel 1 (direction): finishes the previous update's reduction (counts
//            the iteration, tests ||r|| <= rtol ||b||, beta = rho_new / rho);
//            p = D^-1 r + beta p_old, computed on the fly for the tile and its
//            halo; stores p; partials of sigma = p.Ap.
//   kernel 2 (update):    finishes sigma (alpha = rho / sigma, or a
//            breakdown); q = A p recomputed from p (cheaper than storing and
//            re-reading q); r = r - alpha q; partials of r.r (and r.z =
//            sum dinv r^2 for a variable Jacobi scale). x advances every
//            second iteration: odd iterations leave it, even ones add
//            alpha_prev p_prev + alpha p (p_prev is still in the other p
//            buffer); a run that ends after an odd iteration adds the last
//            alpha p with k_x_finish.
//
// Each kernel finishes the reduction its predecessor left (chained
// reductions: no finishing kernel between them); a run of iterations ends
// with a one-wavefront closing kernel for the last update's partials.
//
// p ping-pongs between two buffers: kernel 1 reads halo points of p_old that
// neighbouring work-groups are overwriting in the same launch otherwise.
// With variable coefficients (od.kc) the stencil is the harmonic-mean
// operator and D^-1 is the array od.dinv.
#include <algorithm>

#include "zkernel.hpp"

namespace pcgmi {

namespace {

// Launch of one chained iteration kernel (NC own partials, NCP consumed).
template <int FAM, typename C, class SP, int BX, int BY, int VX, int NC, int NCP, class L, class O, class FP>
hipError_t run_chain(const Geometry& g, const L& ld, const O& op, const FP& fp, const Chain& ch, hipStream_t s) {
    if (g.nblocks == 0) return hipSuccess;
    const dim3 grid(g.nblocks), block(BX * BY);
    if constexpr (FAM == 0)
        hipLaunchKernelGGL((k_pcg_direction<C, SP, BX, BY, VX, NC, NCP, L, O, FP>), grid, block, 0, s, g, ld, op, fp, ch);
    else if constexpr (FAM == 1)
        hipLaunchKernelGGL((k_pcg_update<C, SP, BX, BY, VX, NC, NCP, L, O, FP>), grid, block, 0, s, g, ld, op, fp, ch);
    else
        hipLaunchKernelGGL((k_pcg_sr<C, SP, BX, BY, VX, NC, NCP, L, O, FP>), grid, block, 0, s, g, ld, op, fp, ch);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pcg_direction(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* r,
                                const void* pold, void* pnew, const Chain& ch, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            OpDirection<T, VX> op{static_cast<T*>(pnew)};
            if (od.kc) {
                if constexpr (VAR_TYPE<T>) {
                    LoadDirectionVar<T> ld{static_cast<const T*>(r), static_cast<const T*>(pold),
                                           static_cast<const T*>(od.dinv), od.kc, nullptr, C(0)};
                    return run_chain<0, C, StencilVar<C>, BX, BY, VX, 1, 2>(g, ld, op, FinBeta{nullptr, nullptr, true},
                                                                           ch, s);
                }
                return hipErrorInvalidValue;
            }
            LoadDirection<T> ld{static_cast<const T*>(r), static_cast<const T*>(pold), nullptr, C(0), C(0)};
            return run_chain<0, C, StencilConst<C>, BX, BY, VX, 1, 1>(g, ld, op, FinBeta{nullptr, nullptr, false}, ch,
                                                                     s);
        });
    });
}

hipError_t launch_pcg_update(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* pdir, void* x,
                             int xdt, void* r, int xmode, const void* pprev, const Chain& ch, hipStream_t s) {
    if (xmode != 1 && xmode != 2) return hipErrorInvalidValue;
    // r, p, p_old and x of one iteration against the last-level cache
    const size_t footprint = (size_t)g.nx * g.ny * g.nz * (3 * dt_size(dt) + dt_size(xdt));
    const bool ntx = footprint > LLC_BYTES;
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            // NTX is compiled for the FP64 accumulator only (the widest x stream).
            auto go_x = [&]<bool NTX, int XM>(auto xtag) -> hipError_t {
                using X = decltype(xtag);
                if (od.kc) {
                    if constexpr (VAR_TYPE<T>) {
                        LoadUK<T> ld{static_cast<const T*>(pdir), od.kc};
                        OpUpdate<T, X, VX, true, NTX, XM> op{static_cast<X*>(x), static_cast<T*>(r), nullptr,
                                                             static_cast<const T*>(od.dinv), C(0), 0.0};
                        op.pprev = static_cast<const T*>(pprev);
                        return run_chain<1, C, StencilVar<C>, BX, BY, VX, 2, 1>(g, ld, op, FinAlpha{nullptr}, ch, s);
                    }
                    return hipErrorInvalidValue;
                }
                LoadField<T> ld{static_cast<const T*>(pdir)};
                OpUpdate<T, X, VX, false, NTX, XM> op{static_cast<X*>(x), static_cast<T*>(r), nullptr, nullptr, C(0),
                                                      0.0};
                op.pprev = static_cast<const T*>(pprev);
                return run_chain<1, C, StencilConst<C>, BX, BY, VX, 1, 1>(g, ld, op, FinAlpha{nullptr}, ch, s);
            };
            auto go_nt = [&]<bool NTX>(auto xtag) -> hipError_t {
                if (xmode == 2) return go_x.template operator()<NTX, 2>(xtag);
                // x is not touched: one instantiation serves every accumulator type
                return go_x.template operator()<false, 1>(float{});
            };
            auto go = [&](auto xtag) -> hipError_t {
                using X = decltype(xtag);
                if constexpr (std::is_same_v<X, double>)
                    if (ntx) return go_nt.template operator()<true>(xtag);
                return go_nt.template operator()<false>(xtag);
            };
            if (xdt == DT_F64) return go(double{});
            if (xdt == DT_F32) return go(float{});
            if (xdt == dt) return go(T{});
            return hipErrorInvalidValue;
        });
    });
}

namespace {

// x += alpha p over n points, alpha the state's (rounded to the compute type,
// as the update kernel uses it): the step a run that ends after an odd
// iteration still owes x, or every iteration's step when x must be current
// after each one. check_done: skip when the state records a finished solve
// (the update before it did not run).
template <typename T, typename X>
__global__ void __launch_bounds__(256) k_x_finish(int64_t n, X* __restrict__ x, const T* __restrict__ p,
                                                  const SolveState* st, int check_done) {
    if (check_done && st->done != 0) return;
    using C = typename Traits<T>::C;
    const double a = (double)(C)st->alpha;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = (double)to_c(x[i]) + a * (double)to_c(p[i]);
        st_any<X, 1>(x, i, &v);
    }
}

}  // namespace

hipError_t launch_x_finish(int dt, int xdt, int64_t n, void* x, const void* p, const SolveState* st,
                           bool check_done, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        auto go = [&](auto xtag) -> hipError_t {
            using X = decltype(xtag);
            hipLaunchKernelGGL((k_x_finish<T, X>), dim3((unsigned)blocks), dim3(256), 0, s, n, static_cast<X*>(x),
                               static_cast<const T*>(p), st, check_done ? 1 : 0);
            return hipGetLastError();
        };
        if (xdt == DT_F64) return go(double{});
        if (xdt == DT_F32) return go(float{});
        if (xdt == dt) return go(T{});
        return hipErrorInvalidValue;
    });
}

hipError_t launch_pcg_close(bool var, const Chain& ch, hipStream_t s) {
    if (var) hipLaunchKernelGGL((k_pcg_close<2, FinBeta>), dim3(1), dim3(64), 0, s, FinBeta{nullptr, nullptr, true}, ch);
    else hipLaunchKernelGGL((k_pcg_close<1, FinBeta>), dim3(1), dim3(64), 0, s, FinBeta{nullptr, nullptr, false}, ch);
    return hipGetLastError();
}

hipError_t launch_pcg_sr_start(int dt, const Plan& p, const Geometry& g, const void* r, void* w, SolveState* st,
                               Red red, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            LoadPrecond<T> ld{static_cast<const T*>(r), st, C(0)};
            OpSRStart<T, VX> op{static_cast<const T*>(r), static_cast<T*>(w)};
            return run_zmarch<ZF_SR_START, C, StencilConst<C>, BX, BY, VX, 2, 0u, true>(g, ld, op, FinSRStart{st}, red,
                                                                                      &st->done, s);
        });
    });
}

hipError_t launch_pcg_sr(int dt, const Plan& p, const Geometry& g, const SRBufs& b, void* x, int xdt, const Chain& ch,
                         hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            auto go = [&](auto xtag) -> hipError_t {
                using X = decltype(xtag);
                LoadSR<T> ld{static_cast<const T*>(b.r_in), static_cast<const T*>(b.w_in),
                             static_cast<const T*>(b.s_in), nullptr, C(0), C(0), C(0)};
                OpSR<T, X, VX> op{static_cast<const T*>(b.r_in), static_cast<const T*>(b.w_in),
                                  static_cast<const T*>(b.s_in), static_cast<T*>(b.r_out), static_cast<T*>(b.w_out),
                                  static_cast<T*>(b.s_out), static_cast<T*>(b.p), static_cast<X*>(x), nullptr,
                                  C(0), C(0), C(0), 0.0};
                return run_chain<2, C, StencilConst<C>, BX, BY, VX, 3, 3>(g, ld, op, FinSR{nullptr, nullptr}, ch, s);
            };
            if (xdt == DT_F64) return go(double{});
            if (xdt == DT_F32) return go(float{});
            if (xdt == dt) return go(T{});
            return hipErrorInvalidValue;
        });
    });
}

hipError_t launch_pcg_sr_close(const Chain& ch, hipStream_t s) {
    hipLaunchKernelGGL((k_pcg_close<3, FinSR>), dim3(1), dim3(64), 0, s, FinSR{nullptr, nullptr}, ch);
    return hipGetLastError();
}

hipError_t launch_pcg_start_x0(int dt, int xdt, const Plan& pres, const Geometry& gres, OpDesc od, const void* b,
                               const void* x0, void* r, SolveState* st, double* hist, Red red, hipStream_t s) {
    const int cfg = TILE_CFGS[pres.cfg].vec ? 2 : 5;
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        return dispatch_dt(xdt, [&](auto xtag) {
            using X = decltype(xtag);
            return dispatch_cfg_f64(cfg, [&]<int BX, int BY, int VX>() {
                OpInitResidual<T, VX> op{static_cast<const T*>(b), static_cast<T*>(r),
                                         static_cast<const T*>(od.dinv), st, 0.0};
                if (od.kc) {
                    LoadWidenUK<X, double> ld{static_cast<const X*>(x0), od.kc};
                    return run_zmarch<ZF_START_X0, double, StencilVar<double>, BX, BY, VX, 3, 0u, true>(
                        gres, ld, op, FinStart{st, hist}, red, nullptr, s);
                }
                LoadWiden<X, double> ld{static_cast<const X*>(x0)};
                return run_zmarch<ZF_START_X0, double, StencilConst<double>, BX, BY, VX, 3, 0u, true>(
                    gres, ld, op, FinStart{st, hist}, red, nullptr, s);
            });
        });
    });
}

}  // namespace pcgmi
