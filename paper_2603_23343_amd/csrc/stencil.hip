// stencil.hip -- y = A x (paper Sec. VI) and the FP64 true residual
// r = b - A x with ||r||^2 and max |r|.
#include "zkernel.hpp"

namespace pcgmi {

hipError_t launch_stencil(int dt, const Plan& p, const Geometry& g, const void* x, void* y, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        using C = typename Traits<T>::C;
        return dispatch_cfg<Traits<T>::W>(p.cfg, [&]<int BX, int BY, int VX>() {
            LoadField<T> ld{static_cast<const T*>(x)};
            OpStore<T, VX> op{static_cast<T*>(y)};
            return run_zmarch<ZF_STENCIL, C, BX, BY, VX, 1, 0u, false>(g, ld, op, FinNone{}, Red{nullptr, nullptr}, nullptr, s);
        });
    });
}

// The residual kernel computes in FP64 whatever the storage types, so it
// uses the 128 x 4 double-precision shape (64 x 4 threads, two points each),
// or the scalar shape when nx is odd.
hipError_t launch_residual64(int bdt, int xdt, const Plan& p, const Geometry& g, const void* b, const void* x,
                             double* out, Red red, hipStream_t s) {
    const int cfg = TILE_CFGS[p.cfg].vec ? 2 : 5;
    return dispatch_dt(bdt, [&](auto btag) {
        using B = decltype(btag);
        return dispatch_dt(xdt, [&](auto xtag) {
            using X = decltype(xtag);
            return dispatch_cfg<2>(cfg, [&]<int BX, int BY, int VX>() {
                LoadWiden<X, double> ld{static_cast<const X*>(x)};
                OpResidual64<B, VX> op{static_cast<const B*>(b)};
                return run_zmarch<ZF_RESIDUAL64, double, BX, BY, VX, 2, 2u, true>(g, ld, op, FinStore2{out}, red, nullptr, s);
            });
        });
    });
}

}  // namespace pcgmi
