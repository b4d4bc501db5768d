// refine.hip -- the FP64 pieces of mixed-precision iterative refinement
// (Wilkinson 1963; Moler 1967) around the reduced-precision Jacobi-PCG:
//   cast:    rhat = lp(s (b - A x)), the residual recomputed in FP64 by the
//            z-march stencil and scaled by s = 1 / max|r| before rounding, so
//            16-bit storage keeps its full relative precision;
//   correct: x += d / s in FP64, d the inner solution (storage type or FP64).
#include "zkernel.hpp"

namespace pcgmi {

namespace {

template <typename D>
__global__ void __launch_bounds__(STREAM_THREADS) k_correct(int64_t n, const D* __restrict__ d, double scale,
                                                            double* __restrict__ x) {
    const int64_t stride = (int64_t)gridDim.x * STREAM_THREADS;
    for (int64_t i = (int64_t)blockIdx.x * STREAM_THREADS + threadIdx.x; i < n; i += stride)
        x[i] += (double)to_c(d[i]) / scale;
}

}  // namespace

hipError_t launch_cast_scaled(int dt, const Plan& pres, const Geometry& gres, OpDesc od, const double* b,
                              const double* x, double scale, void* rhat, hipStream_t s) {
    const int cfg = TILE_CFGS[pres.cfg].vec ? 2 : 5;
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        return dispatch_cfg_f64(cfg, [&]<int BX, int BY, int VX>() {
            OpCastScaled<T, VX> op{b, static_cast<T*>(rhat), scale};
            if (od.kc) {
                LoadWidenUK<double, double> ld{x, od.kc};
                return run_zmarch<ZF_GENERIC, double, StencilVar<double>, BX, BY, VX, 1, 0u, false>(
                    gres, ld, op, FinNone{}, Red{nullptr, nullptr, 0}, nullptr, s);
            }
            LoadWiden<double, double> ld{x};
            return run_zmarch<ZF_GENERIC, double, StencilConst<double>, BX, BY, VX, 1, 0u, false>(
                gres, ld, op, FinNone{}, Red{nullptr, nullptr, 0}, nullptr, s);
        });
    });
}

hipError_t launch_correct(int ddt, int64_t n, const void* d, double scale, double* x, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return dispatch_dt(ddt, [&](auto tag) {
        using D = decltype(tag);
        int64_t nb = (n + STREAM_THREADS * 4 - 1) / (STREAM_THREADS * 4);
        nb = nb < 1 ? 1 : (nb > 8192 ? 8192 : nb);
        hipLaunchKernelGGL(k_correct<D>, dim3((unsigned)nb), dim3(STREAM_THREADS), 0, s, n,
                           static_cast<const D*>(d), scale, x);
        return hipGetLastError();
    });
}

}  // namespace pcgmi
