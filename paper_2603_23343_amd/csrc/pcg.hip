// pcg.hip -- the two fused kernels of one Jacobi-PCG iteration (paper
// Sec. VII composes PCG from the stencil, the dot reduction and element-wise
// updates; here they are fused so each iteration makes two passes over HBM):
//
//   kernel 1 (direction): p = D^-1 r + beta p_old, computed on the fly for the
//            tile and its halo; stores p; sigma = p.Ap; the last work-group
//            forms alpha = rho / sigma (or flags a breakdown).
//   kernel 2 (update):    q = A p recomputed from p (cheaper than storing and
//            re-reading q); x += alpha p; r = r - alpha q; rr = r.r (and
//            r.z = sum dinv r^2 for a variable Jacobi scale); the last
//            work-group counts the iteration, tests ||r|| <= rtol ||b|| and
//            forms beta = rho_new / rho.
//
// p ping-pongs between two buffers: kernel 1 reads halo points of p_old that
// neighbouring work-groups are overwriting in the same launch otherwise.
// With variable coefficients (od.kc) the stencil is the harmonic-mean
// operator and D^-1 is the array od.dinv.
#include "zkernel.hpp"

namespace pcgmi {

hipError_t launch_pcg_direction(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* r,
                                const void* pold, void* pnew, SolveState* st, Red red, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            OpDirection<T, VX> op{static_cast<T*>(pnew)};
            if (od.kc) {
                if constexpr (VAR_TYPE<T>) {
                    LoadDirectionVar<T> ld{static_cast<const T*>(r), static_cast<const T*>(pold),
                                           static_cast<const T*>(od.dinv), od.kc, st, C(0)};
                    return run_zmarch<ZF_DIRECTION, C, StencilVar<C>, BX, BY, VX, 1, 0u, true>(
                        g, ld, op, FinAlpha{st}, red, &st->done, s);
                }
                return hipErrorInvalidValue;
            }
            LoadDirection<T> ld{static_cast<const T*>(r), static_cast<const T*>(pold), st, C(0), C(0)};
            return run_zmarch<ZF_DIRECTION, C, StencilConst<C>, BX, BY, VX, 1, 0u, true>(g, ld, op, FinAlpha{st},
                                                                                         red, &st->done, s);
        });
    });
}

hipError_t launch_pcg_update(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* pdir, void* x,
                             int xdt, void* r, SolveState* st, double* hist, Red red, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            auto go = [&](auto xtag) -> hipError_t {
                using X = decltype(xtag);
                if (od.kc) {
                    if constexpr (VAR_TYPE<T>) {
                        LoadUK<T> ld{static_cast<const T*>(pdir), od.kc};
                        OpUpdate<T, X, VX, true> op{static_cast<X*>(x), static_cast<T*>(r), st,
                                                    static_cast<const T*>(od.dinv), C(0), 0.0};
                        return run_zmarch<ZF_UPDATE, C, StencilVar<C>, BX, BY, VX, 2, 0u, true>(
                            g, ld, op, FinBeta{st, hist, true}, red, &st->done, s);
                    }
                    return hipErrorInvalidValue;
                }
                LoadField<T> ld{static_cast<const T*>(pdir)};
                OpUpdate<T, X, VX> op{static_cast<X*>(x), static_cast<T*>(r), st, nullptr, C(0), 0.0};
                return run_zmarch<ZF_UPDATE, C, StencilConst<C>, BX, BY, VX, 1, 0u, true>(
                    g, ld, op, FinBeta{st, hist, false}, red, &st->done, s);
            };
            if (xdt == DT_F64) return go(double{});
            if (xdt == DT_F32) return go(float{});
            if (xdt == dt) return go(T{});
            return hipErrorInvalidValue;
        });
    });
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
