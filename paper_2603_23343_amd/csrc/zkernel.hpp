// zkernel.hpp -- the generic z-march kernel and the dispatch over storage
// types and compiled work-group shapes.
#pragma once

#include <type_traits>

#include "ops.hpp"

namespace pcgmi {

// One work-group per (x-y tile, z chunk). NC reduction components are
// combined over the grid (component c maxed when bit c of MM is set) and
// handed to fin, either by the last work-group (atomic ticket) or, with
// split, by a one-work-group finishing kernel launched next: every
// work-group's agent-scope release fence costs ~40 ns of serialized time on
// this multi-XCD part (measured), which a kernel boundary replaces. Both ways
// sum the partials in the same order. A set *done skips the launch's work:
// captured PCG iterations after convergence cost only the launch.
template <typename C, class SP, int BX, int BY, int VX, int NC, unsigned MM, bool RED, class L, class O, class F>
__device__ __forceinline__ void zmarch_body(const Grid3& g, const L& ld, const O& op, const F& fin, Red red,
                                            const int* done, int split) {
    if (done != nullptr && *done != 0) return;
    using Cell = typename SP::Cell;
    using ZT = ZTile<Cell, BX, BY, VX>;
    __shared__ __attribute__((aligned(16))) Cell lds[2 * ZT::PLANE];
    __shared__ double rscratch[NC * 16];
    L l = ld;
    O o = op;
    l.init();
    o.init();
    const unsigned tile = xcd_remap(blockIdx.x, g.nblocks);
    C acc[NC];
    zmarch<C, SP, BX, BY, VX, NC>(g, tile, l, o, acc, lds);
    if constexpr (RED) {
        double v[NC], tot[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = (double)acc[c];
        if (split) {
            block_reduce<NC, MM>(v, rscratch);
            if (threadIdx.x == 0)
#pragma unroll
                for (int c = 0; c < NC; ++c) red.partials[NC * blockIdx.x + c] = v[c];
            return;
        }
        if (grid_reduce<NC, MM>(v, red.partials, red.ticket, g.nblocks, blockIdx.x, rscratch, tot) &&
            threadIdx.x == 0)
            fin(tot);
    }
}

// The finishing kernel of the split reduction: one work-group of the z-march
// kernel's size sums the partials as the last work-group would, then fin.
template <int NC, unsigned MM, class F>
__global__ void __launch_bounds__(256) k_zfinish(const double* __restrict__ partials, unsigned nblocks, F fin,
                                                 const int* done) {
    if (done != nullptr && *done != 0) return;
    __shared__ double lds[NC * 16];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (unsigned i = threadIdx.x; i < nblocks; i += blockDim.x)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double t = partials[NC * i + c];
            if ((MM >> c) & 1u) acc[c] = t > acc[c] ? t : acc[c];
            else acc[c] += t;
        }
    block_reduce<NC, MM>(acc, lds);
    if (threadIdx.x == 0) fin(acc);
}

// Work-groups from which a reducing z-march splits off its finishing kernel.
constexpr unsigned SPLIT_MIN_BLOCKS = 64;

// One __global__ name per kernel family (so profiles tell them apart), all
// running the same body.
#define PCGMI_ZKERNEL(NAME)                                                                               \
    template <typename C, class SP, int BX, int BY, int VX, int NC, unsigned MM, bool RED, class L, class O, \
              class F>                                                                                    \
    __global__ void __launch_bounds__(BX* BY) NAME(Grid3 g, L ld, O op, F fin, Red red, const int* done,   \
                                                   int split) {                                           \
        zmarch_body<C, SP, BX, BY, VX, NC, MM, RED>(g, ld, op, fin, red, done, split);                    \
    }
PCGMI_ZKERNEL(k_stencil)
PCGMI_ZKERNEL(k_flex_direction)
PCGMI_ZKERNEL(k_residual64)
PCGMI_ZKERNEL(k_start_x0)
PCGMI_ZKERNEL(k_sr_start)
PCGMI_ZKERNEL(k_zgeneric)
PCGMI_ZKERNEL(k_mg_smooth_select)

enum ZFamily { ZF_STENCIL, ZF_FLEX_DIRECTION, ZF_RESIDUAL64, ZF_START_X0, ZF_SR_START, ZF_GENERIC, ZF_MG_SELECT };

template <int FAM, typename C, class SP, int BX, int BY, int VX, int NC, unsigned MM, bool RED, class L, class O,
          class F>
hipError_t run_zmarch(const Grid3& g, const L& ld, const O& op, const F& fin, Red red, const int* done,
                      hipStream_t s) {
    if (g.nblocks == 0) return hipSuccess;
    if (RED && (red.partials == nullptr || (size_t)NC * g.nblocks > red.cap)) return hipErrorInvalidValue;
    const dim3 grid(g.nblocks), block(BX * BY);
    const int split = (RED && g.nblocks >= SPLIT_MIN_BLOCKS) ? 1 : 0;
    if constexpr (FAM == ZF_STENCIL)
        hipLaunchKernelGGL((k_stencil<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    else if constexpr (FAM == ZF_FLEX_DIRECTION)
        hipLaunchKernelGGL((k_flex_direction<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    else if constexpr (FAM == ZF_RESIDUAL64)
        hipLaunchKernelGGL((k_residual64<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    else if constexpr (FAM == ZF_SR_START)
        hipLaunchKernelGGL((k_sr_start<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    else if constexpr (FAM == ZF_START_X0)
        hipLaunchKernelGGL((k_start_x0<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    else if constexpr (FAM == ZF_MG_SELECT)
        hipLaunchKernelGGL((k_mg_smooth_select<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    else
        hipLaunchKernelGGL((k_zgeneric<C, SP, BX, BY, VX, NC, MM, RED, L, O, F>), grid, block, 0, s, g, ld, op, fin, red, done, split);
    if (split) hipLaunchKernelGGL((k_zfinish<NC, MM, F>), dim3(1), block, 0, s, red.partials, g.nblocks, fin, done);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Chained reductions of the PCG iteration kernels. Each iteration kernel
// leaves one partial per work-group (and component); the NEXT kernel on the
// stream finishes that reduction itself instead of a one-work-group kernel in
// between: every work-group sums the partials (wave 0, lanes striding the
// partials in index order, then the fixed butterfly, so every work-group and
// the closing kernel get bit-identical totals whatever their size), applies
// the finisher to its own LDS copy of the solve state and continues with
// those scalars; work-group 0 stores the copy as the next state. The state is
// double-buffered (sin read, sout written) so no work-group reads a state that
// another work-group of the same launch is writing. A done state is passed
// on (copied) and skips the work.
template <class T> __device__ __forceinline__ void bind_state(T& t, SolveState* s) {
    if constexpr (requires { t.st = s; }) t.st = s;
}

// Returns whether the work-group goes on to its own work (uniform).
template <int NCP, class FP>
__device__ __forceinline__ bool chain_enter(const Chain& ch, const FP& fp, SolveState& s_st) {
    // The partials are summed while the state is read (both are loads of the
    // previous kernel's output); a done state discards the sum.
    // Each lane issues eight loads before it adds (a dependent load per add
    // costs one L2 round trip each: 16 of them at 1024 work-groups); the
    // additions keep index order, so the totals do not depend on it.
    constexpr int PU = 8;
    double v[NCP];
#pragma unroll
    for (int c = 0; c < NCP; ++c) v[c] = 0.0;
    if (ch.pin != nullptr && threadIdx.x < 64)
        for (unsigned base = threadIdx.x; base < ch.nin; base += 64 * PU) {
            double t[PU][NCP];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const unsigned i = base + 64 * u;
#pragma unroll
                for (int c = 0; c < NCP; ++c) t[u][c] = i < ch.nin ? ch.pin[NCP * i + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < PU; ++u)
#pragma unroll
                for (int c = 0; c < NCP; ++c) v[c] += t[u][c];
        }
    if (threadIdx.x == 0) s_st = *ch.sin;
    __syncthreads();
    if (s_st.done != 0) {
        if (ch.pin != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *ch.sout = s_st;
        return false;
    }
    if (ch.pin != nullptr) {
        if (threadIdx.x < 64) {
#pragma unroll
            for (int c = 0; c < NCP; ++c) v[c] = wave_sum(v[c]);
            if (threadIdx.x == 0) {
                FP f = fp;
                bind_state(f, &s_st);
                if constexpr (requires { f.hist; }) f.hist = blockIdx.x == 0 ? ch.hist : nullptr;
                f(v);
                if (blockIdx.x == 0) *ch.sout = s_st;
            }
        }
        __syncthreads();
        if (s_st.done != 0) return false;
    }
    return true;
}

template <typename C, class SP, int BX, int BY, int VX, int NC, int NCP, class L, class O, class FP>
__device__ __forceinline__ void chain_body(const Grid3& g, const L& ld, const O& op, const FP& fp, const Chain& ch) {
    using Cell = typename SP::Cell;
    using ZT = ZTile<Cell, BX, BY, VX>;
    __shared__ __attribute__((aligned(16))) Cell lds[2 * ZT::PLANE];
    __shared__ double rscratch[NC * 16];
    __shared__ SolveState s_st;
    if (!chain_enter<NCP>(ch, fp, s_st)) return;
    L l = ld;
    O o = op;
    bind_state(l, &s_st);
    bind_state(o, &s_st);
    l.init();
    o.init();
    const unsigned tile = xcd_remap(blockIdx.x, g.nblocks);
    C acc[NC];
    zmarch<C, SP, BX, BY, VX, NC>(g, tile, l, o, acc, lds);
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = (double)acc[c];
    block_reduce<NC, 0u>(v, rscratch);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) ch.pout[NC * blockIdx.x + c] = v[c];
}

#define PCGMI_CHAIN_KERNEL(NAME)                                                                          \
    template <typename C, class SP, int BX, int BY, int VX, int NC, int NCP, class L, class O, class FP>  \
    __global__ void __launch_bounds__(BX* BY) NAME(Grid3 g, L ld, O op, FP fp, Chain ch) {                \
        chain_body<C, SP, BX, BY, VX, NC, NCP>(g, ld, op, fp, ch);                                        \
    }
PCGMI_CHAIN_KERNEL(k_pcg_direction)
PCGMI_CHAIN_KERNEL(k_pcg_update)
PCGMI_CHAIN_KERNEL(k_pcg_sr)

// Finishes the last kernel's partials of a run of chained kernels (one wavefront).
template <int NCP, class FP> __global__ void __launch_bounds__(64) k_pcg_close(FP fp, Chain ch) {
    __shared__ SolveState s_st;
    (void)chain_enter<NCP>(ch, fp, s_st);
}

// Calls f.template operator()<BX, BY, VX>() for compiled shape cfg, W being
// the 16-byte vector width of the kernel's storage type.
template <int W, class F> hipError_t dispatch_cfg(int cfg, F&& f) {
    switch (cfg) {
        case 0: return f.template operator()<16, 16, W>();
        case 1: return f.template operator()<32, 8, W>();
        case 2: return f.template operator()<64, 4, W>();
        case 3: return f.template operator()<16, 4, W>();
        case 4: return f.template operator()<16, 8, W>();
        case 5: return f.template operator()<64, 4, 1>();
        default: return hipErrorInvalidValue;
    }
}

// The FP64 residual and start kernels compile only the 64 x 4 shapes
// (cfg 2: two doubles per thread, cfg 5: one).
template <class F> hipError_t dispatch_cfg_f64(int cfg, F&& f) {
    switch (cfg) {
        case 2: return f.template operator()<64, 4, 2>();
        case 5: return f.template operator()<64, 4, 1>();
        default: return hipErrorInvalidValue;
    }
}

// Storage types with variable-coefficient kernels compiled.
template <typename T> constexpr bool VAR_TYPE = std::is_same_v<T, float> || std::is_same_v<T, double>;

// Calls f(T{}) with T the storage type of dt.
template <class F> hipError_t dispatch_dt(int dt, F&& f) {
    switch (dt) {
        case DT_F32: return f(float{});
        case DT_BF16: return f(bf16{});
        case DT_F16: return f(_Float16{});
        case DT_F64: return f(double{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pcgmi
