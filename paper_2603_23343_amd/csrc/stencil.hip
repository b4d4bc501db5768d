// stencil.hip -- y = A x (paper Sec. VI), constant or variable coefficients,
// the FP64 true residual r = b - A x with ||r||^2 and max |r|, and the
// inverse diagonal of the variable-coefficient operator.
#include <type_traits>

#include "zkernel.hpp"

namespace pcgmi {

hipError_t launch_stencil(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* x, void* y, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            OpStore<T, VX> op{static_cast<T*>(y)};
            if (od.kc) {
                if constexpr (VAR_TYPE<T>) {
                    LoadUK<T> ld{static_cast<const T*>(x), od.kc};
                    return run_zmarch<ZF_STENCIL, C, StencilVar<C>, BX, BY, VX, 1, 0u, false>(
                        g, ld, op, FinNone{}, Red{nullptr, nullptr, 0}, nullptr, s);
                }
                return hipErrorInvalidValue;
            }
            LoadField<T> ld{static_cast<const T*>(x)};
            return run_zmarch<ZF_STENCIL, C, StencilConst<C>, BX, BY, VX, 1, 0u, false>(
                g, ld, op, FinNone{}, Red{nullptr, nullptr, 0}, nullptr, s);
        });
    });
}

// The residual kernel computes in FP64 whatever the storage types, so it
// uses the 128 x 4 double-precision shape (64 x 4 threads, two points each),
// or the scalar shape when nx is odd.
hipError_t launch_residual64(int bdt, int xdt, const Plan& p, const Geometry& g, OpDesc od, const void* b,
                             const void* x, double* out, Red red, hipStream_t s) {
    const int cfg = TILE_CFGS[p.cfg].vec ? 2 : 5;
    return dispatch_dt(bdt, [&](auto btag) {
        using B = decltype(btag);
        return dispatch_dt(xdt, [&](auto xtag) {
            using X = decltype(xtag);
            return dispatch_cfg_f64(cfg, [&]<int BX, int BY, int VX>() {
                OpResidual64<B, VX> op{static_cast<const B*>(b)};
                if (od.kc) {
                    LoadWidenUK<X, double> ld{static_cast<const X*>(x), od.kc};
                    return run_zmarch<ZF_RESIDUAL64, double, StencilVar<double>, BX, BY, VX, 2, 2u, true>(
                        g, ld, op, FinStore2{out}, red, nullptr, s);
                }
                LoadWiden<X, double> ld{static_cast<const X*>(x)};
                return run_zmarch<ZF_RESIDUAL64, double, StencilConst<double>, BX, BY, VX, 2, 2u, true>(
                    g, ld, op, FinStore2{out}, red, nullptr, s);
            });
        });
    });
}

hipError_t launch_var_dinv(int dt, const Plan& p, const Geometry& g, const float* kc, void* dinv, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        if constexpr (VAR_TYPE<T>) {
            return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
                LoadK<C> ld{kc};
                OpStoreInverse<T, VX> op{static_cast<T*>(dinv)};
                return run_zmarch<ZF_GENERIC, C, StencilVarDiag<C>, BX, BY, VX, 1, 0u, false>(
                    g, ld, op, FinNone{}, Red{nullptr, nullptr, 0}, nullptr, s);
            });
        }
        return hipErrorInvalidValue;
    });
}

}  // namespace pcgmi
