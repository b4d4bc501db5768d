// batched.hip -- many independent Jacobi-PCG solves (the paper's Sec. VII
// solver on grids of different sizes) in ONE persistent launch.
//
// Every work-group of the launch belongs to one problem. A problem owns a
// group of work-groups, all on one XCD: the dispatcher deals work-groups to
// the 8 XCDs round-robin (from some starting XCD), so a group is a set of
// blocks with the same b mod 8 and shares that XCD's L2; the kernel checks
// this with the hardware XCD id before relying on it.
// The group runs the same two fused iteration phases as the single-problem
// solver (direction: p = D^-1 r + beta p_old, sigma = p.Ap; update: x +=
// alpha p, r -= alpha Ap, r.r) over its problem's tiles, separated by group
// barriers. Reductions: each work-group writes its partial, the barrier
// publishes them, and every work-group of the group sums all partials of its
// group in rank order, so all members hold bit-identical scalars and stop
// together. Partials alternate between two buffers so a fast work-group
// writing the next phase's partials never overwrites ones a slow one is
// still reading.
//
// The launch is sized to the device's resident capacity (occupancy x CUs),
// so every group's work-groups run concurrently; every barrier wait is
// bounded (a spin limit sets an error flag and the work-group leaves), so the
// kernel always terminates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "trace.hpp"
#include "zkernel.hpp"

namespace pcgmi {
const char* set_error(pcg_status st, const char* msg);
}

namespace pcgmi {

struct BatchProb {
    int64_t off;   // element offset of the problem in the caller's b and x arenas
    int64_t ioff;  // element offset in the internal (row-padded) arenas
    int nx, ny, nz;
    int pitch;     // internal row stride: nx rounded up to 4
    int cfg, zc;
    int ntx, nty, nzc, ntiles;
    int group;     // work-groups of the problem
    int pad;
};

struct BatchOut {
    int iters;
    int done;      // 1 converged, 2 breakdown, 3 maxit
    int restarts;  // FP64 residual restarts taken
    int xcd_local; // group barriers ran in the XCD-local form
    double rr, rr0, rr_true;  // recursive ||r||^2, ||b||^2, FP64 ||b - A x||^2
    unsigned long long t_begin, t_done;
};

// Restarts from the FP64 residual per problem at most (default).
constexpr int BATCH_MAX_RESTARTS = 3;

namespace {

constexpr int BT = 256;                 // threads per work-group (all shapes below)
constexpr long long SPIN_LIMIT = 1 << 22;  // ~0.2 s of s_sleep(2) per barrier wait

// Per-problem barrier words, one 128-byte line per problem: arrival count,
// generation, and the mask of XCDs its members run on.
constexpr int BAR_WORDS = 32;

// XCD (XCC) of the calling wavefront, from the hardware register XCC_ID.
__device__ __forceinline__ unsigned xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu; }

// Group barrier: count arrivals; the last arrival resets the count and bumps
// the generation; the others wait (bounded) for the bump.
// Visibility of the group's global writes (directions, residuals, partials):
//  - general form: agent-scope release / acquire fences (an L2 write-back
//    per work-group, ~40 ns of serialized device time each on MI355X);
//  - XCD-local form, when every member runs on one XCD (the XCD mask of the
//    group, gathered at the start, has one bit): the members share that
//    XCD's L2, so it is enough that
//    every wavefront's stores have completed (s_waitcnt 0) before the arrival
//    atomic, and that readers drop their L1 contents (agent-scope acquire)
//    after the generation changes. 1.7x faster on the 64-problem batch.
__device__ __forceinline__ bool group_barrier(unsigned* cnt, unsigned* gen, unsigned nwg, unsigned& my_gen,
                                              int* err, bool xcd_local) {
    __shared__ int s_ok;
    if (xcd_local) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        if (!xcd_local) __threadfence();
        const unsigned a = atomicAdd(cnt, 1u);
        if (a == nwg - 1) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (xcd_local) __builtin_amdgcn_s_waitcnt(0);
            else __threadfence();
            atomicAdd(gen, 1u);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == my_gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > SPIN_LIMIT || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    atomicExch(err, 1);
                    break;
                }
            }
        }
        if (xcd_local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        else __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    ++my_gen;
    return s_ok != 0;
}

// Sum of the group's partials in rank order (every member gets the same bits).
__device__ __forceinline__ double group_sum(const double* part, int G, double* lds) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < G; i += BT)
        v[0] += __hip_atomic_load(&part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    block_reduce<1, 0u>(v, lds);
    __shared__ double s_tot;
    if (threadIdx.x == 0) s_tot = v[0];
    __syncthreads();
    return s_tot;
}

// One z-march over tile t of a problem with the shape selected at run time.
template <class LF, class OF>
__device__ __forceinline__ float march(const BatchProb& pr, unsigned t, LF&& mkld, OF&& mkop, float* lds) {
    Geometry g{pr.nx, pr.ny, pr.nz, pr.ntx, pr.nty, pr.nzc, pr.zc, (unsigned)pr.ntiles, pr.pitch};
    float acc[1] = {0.f};
    switch (pr.cfg) {
        case 0: zmarch<float, StencilConst<float>, 16, 16, 4, 1, true>(g, t, mkld(), mkop.template operator()<4>(), acc, lds); break;
        case 1: zmarch<float, StencilConst<float>, 32, 8, 4, 1, true>(g, t, mkld(), mkop.template operator()<4>(), acc, lds); break;
        case 2: zmarch<float, StencilConst<float>, 64, 4, 4, 1, true>(g, t, mkld(), mkop.template operator()<4>(), acc, lds); break;
        default: zmarch<float, StencilConst<float>, 64, 4, 1, 1>(g, t, mkld(), mkop.template operator()<1>(), acc, lds); break;
    }
    __syncthreads();  // the next tile restages the same LDS planes
    return acc[0];
}

// FP64 true residual of the group's problem over a contiguous range of
// points per work-group: r = fl32(b - A x) (the restart residual), and the
// work-group's sums of (b - A x)^2 and of the stored r^2. b is in the
// caller's layout, x and r in the row-padded one. With po, x still owes the
// step a_owed po (x advances every second iteration): the residual is that
// of x + a_owed po, formed on the fly exactly as the step will be stored.
__device__ __forceinline__ void true_residual(const BatchProb& pr, const float* __restrict__ b,
                                              const double* __restrict__ x, const float* __restrict__ po,
                                              double a_owed, float* __restrict__ r, int rank, int G, double& rrt,
                                              double& rrs) {
    const unsigned nx = pr.nx, ny = pr.ny, nz = pr.nz, n = nx * ny * nz, sy = pr.pitch, sz = sy * ny;
    const unsigned per = (n + G - 1) / G, lo = (unsigned)rank * per, hi = min(lo + per, n);
    rrt = 0.0;
    rrs = 0.0;
    for (unsigned i = lo + threadIdx.x; i < hi; i += BT) {
        const unsigned ix = i % nx, row = i / nx, iy = row % ny, iz = row / ny;
        const unsigned j = row * sy + ix;
        auto xe = [&](unsigned k) { return po ? x[k] + a_owed * (double)po[k] : x[k]; };
        double ax = 6.0 * xe(j);
        if (ix > 0) ax -= xe(j - 1);
        if (ix + 1 < nx) ax -= xe(j + 1);
        if (iy > 0) ax -= xe(j - sy);
        if (iy + 1 < ny) ax -= xe(j + sy);
        if (iz > 0) ax -= xe(j - sz);
        if (iz + 1 < nz) ax -= xe(j + sz);
        const double res = (double)b[i] - ax;
        const float rf = (float)res;
        r[j] = rf;
        rrt += res * res;
        rrs += (double)rf * (double)rf;
    }
}

// Publish a work-group's components (thread 0 holds the block sums) to
// slots [c * maxg + rank] of a partials buffer.
template <int NC>
__device__ __forceinline__ void put_partials(double (&v)[NC], double* part, int maxg, int rank, double* rs) {
    block_reduce<NC, 0u>(v, rs);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            __hip_atomic_store(&part[c * maxg + rank], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Partials per problem: three buffers of two components x maxg slots. The
// direction phase uses A, the update phase B, the start and the FP64
// residual steps C: a buffer is rewritten only after a barrier that every
// reader of its previous contents has passed.
__global__ void __launch_bounds__(BT, 3) k_batch_pcg(const BatchProb* __restrict__ probs, const int2* __restrict__ wgmap,
                                                   const float* __restrict__ b, double* __restrict__ x, float* r,
                                                   float* p0, float* p1, double* xacc, double* partials, int maxg,
                                                   int part_stride, unsigned* bar,
                                                   BatchOut* out, double rtol2, int maxit, int* err,
                                                   int force_agent, int max_restarts) {
    __shared__ __attribute__((aligned(16))) float lds[3168];
    __shared__ double rs[32];
    const int2 m = wgmap[blockIdx.x];
    if (m.x < 0) return;
    const int pi = m.x, rank = m.y;
    const BatchProb pr = probs[pi];
    const int G = pr.group;
    unsigned* cnt = bar + BAR_WORDS * pi;
    unsigned* gen = cnt + 1;
    unsigned* xcd_mask = cnt + 2;
    double* partA = partials + (size_t)pi * part_stride;
    double* partB = partA + 2 * maxg;
    double* partC = partA + 4 * maxg;
    unsigned my_gen = 0;
    const float* bp = b + pr.off;
    double* xp = xacc + pr.ioff;
    float* rp = r + pr.ioff;
    float* pp[2] = {p0 + pr.ioff, p1 + pr.ioff};
    const unsigned long long t_begin = wall_clock64();
    // The dispatcher deals work-groups to the XCDs round-robin, so members
    // (blocks with the same b mod 8) should share one; record where they run.
    if (threadIdx.x == 0) atomicOr(xcd_mask, 1u << xcc_id());

    // Start (row-padded layout, padding 0): r = b, x = 0, p0 = 0; ||b||^2.
    double bb = 0.0;
    {
        const unsigned nxp = pr.pitch, npad = nxp * pr.ny * pr.nz;
        const unsigned per = (npad + G - 1) / G, lo = (unsigned)rank * per, hi = min(lo + per, npad);
        float acc = 0.f;
        for (unsigned j = lo + threadIdx.x; j < hi; j += BT) {
            const unsigned ix = j % nxp, row = j / nxp;
            const float bv = ix < (unsigned)pr.nx ? bp[row * pr.nx + ix] : 0.f;
            rp[j] = bv;
            pp[0][j] = 0.f;
            xp[j] = 0.0;
            acc += bv * bv;
        }
        double v[1] = {(double)acc};
        put_partials<1>(v, partC, maxg, rank, rs);
        if (!group_barrier(cnt, gen, G, my_gen, err, false)) return;
        bb = group_sum(partC, G, rs);
    }
    // every member reads the flag after the same barrier: one decision per group
    // (force_agent keeps the general form even for a group on one XCD)
    const bool xl = !force_agent &&
                    __popc(__hip_atomic_load(xcd_mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 1;
    const double tol2 = rtol2 * bb;
    double rho = bb / 6.0, beta = 0.0, rr = bb, rrt = bb;
    int it = 0, restarts = 0, done = 0, io = 0;
    // x advances every second update: after one that left it, x owes
    // alpha_owed p (p still in its buffer), added by the next update
    // together with that update's own step, or at a stop of the recursion.
    bool x_owed = false;
    float alpha_owed = 0.f;
    // Store the owed step on this work-group's points (the true residual's
    // range, the same threads as the copy to the caller's layout below).
    auto settle_x = [&]() {
        if (!x_owed) return;
        const unsigned nx = pr.nx, n = nx * pr.ny * pr.nz;
        const unsigned per = (n + G - 1) / G, lo = (unsigned)rank * per, hi = min(lo + per, n);
        const float* po = pp[io];
        for (unsigned i = lo + threadIdx.x; i < hi; i += BT) {
            const unsigned j = (i / nx) * pr.pitch + i % nx;
            xp[j] = xp[j] + (double)alpha_owed * (double)po[j];
        }
        x_owed = false;
    };
    if (!isfinite(bb)) done = 2;
    else if (bb == 0.0) done = 1;
    while (!done) {
        float* pold = pp[io];
        float* pnew = pp[io ^ 1];
        // Phase 1: direction and sigma = p.Ap.
        float acc = 0.f;
        for (int t = rank; t < pr.ntiles; t += G) {
            acc += march(
                pr, (unsigned)t,
                [&]() {
                    LoadDirection<float> l{rp, pold, nullptr, (float)beta, 1.f / 6.f};
                    return l;
                },
                [&]<int VX>() { return OpDirection<float, VX>{pnew}; }, lds);
        }
        {
            double v[1] = {(double)acc};
            put_partials<1>(v, partA, maxg, rank, rs);
        }
        if (!group_barrier(cnt, gen, G, my_gen, err, xl)) return;
        const double sigma = group_sum(partA, G, rs);
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            done = 2;
            break;
        }
        const float alpha = (float)(rho / sigma);
        // Phase 2: update and r.r; x takes two steps every second update.
        acc = 0.f;
        if (x_owed) {
            for (int t = rank; t < pr.ntiles; t += G) {
                acc += march(
                    pr, (unsigned)t,
                    [&]() {
                        LoadField<float> l{pnew};
                        return l;
                    },
                    [&]<int VX>() {
                        OpUpdate<float, double, VX, false, false, 2> o{xp, rp, nullptr, nullptr, alpha, (double)alpha};
                        o.pprev = pold;
                        o.alpha_prev_d = (double)alpha_owed;
                        return o;
                    },
                    lds);
            }
        } else {
            for (int t = rank; t < pr.ntiles; t += G) {
                acc += march(
                    pr, (unsigned)t,
                    [&]() {
                        LoadField<float> l{pnew};
                        return l;
                    },
                    [&]<int VX>() {
                        return OpUpdate<float, double, VX, false, false, 1>{xp, rp, nullptr, nullptr, alpha,
                                                                            (double)alpha};
                    },
                    lds);
            }
        }
        x_owed = !x_owed;
        alpha_owed = alpha;
        {
            double v[1] = {(double)acc};
            put_partials<1>(v, partB, maxg, rank, rs);
        }
        if (!group_barrier(cnt, gen, G, my_gen, err, xl)) return;
        rr = group_sum(partB, G, rs);
        ++it;
        io ^= 1;
        if (!isfinite(rr)) {
            done = 2;
            break;
        }
        if (rr > tol2 && it < maxit) {
            const double rho_new = rr / 6.0;
            beta = rho_new / rho;
            rho = rho_new;
            continue;
        }
        // The recursion has stopped: judge by the FP64 true residual and,
        // if it is above the tolerance, restart from x with r = b - A x.
        {
            double v[2];
            true_residual(pr, bp, xp, x_owed ? pp[io] : nullptr, (double)alpha_owed, rp, rank, G, v[0], v[1]);
            put_partials<2>(v, partC, maxg, rank, rs);
        }
        if (!group_barrier(cnt, gen, G, my_gen, err, xl)) return;
        rrt = group_sum(partC, G, rs);
        const double rrs = group_sum(partC + maxg, G, rs);
        // every member has read x past the barrier; the next reads of
        // other work-groups' points come after later barriers
        settle_x();
        if (rrt <= tol2 || rr > tol2 || restarts >= max_restarts || it >= maxit) {
            done = rr <= tol2 ? 1 : 3;
            break;
        }
        ++restarts;
        rr = rrs;
        rho = rrs / 6.0;
        beta = 0.0;
    }
    // a stop on a breakdown can still owe a step
    settle_x();
    // x to the caller's layout (the last update phase is behind a barrier).
    {
        const unsigned nx = pr.nx, n = nx * pr.ny * pr.nz;
        const unsigned per = (n + G - 1) / G, lo = (unsigned)rank * per, hi = min(lo + per, n);
        double* xo = x + pr.off;
        for (unsigned i = lo + threadIdx.x; i < hi; i += BT) xo[i] = xp[(i / nx) * pr.pitch + i % nx];
    }
    if (rank == 0 && threadIdx.x == 0) {
        BatchOut o;
        o.iters = it;
        o.done = done;
        o.restarts = restarts;
        o.xcd_local = xl ? 1 : 0;
        o.rr = rr;
        o.rr0 = bb;
        o.rr_true = rrt;
        o.t_begin = t_begin;
        o.t_done = wall_clock64();
        out[pi] = o;
    }
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct BatchImpl {
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    int nprob = 0;
    std::vector<BatchProb> probs;
    std::vector<int2> wgmap;
    std::vector<int> cap_tiles;  // upper bound on a problem's tile count
    int grid = 0, maxg = 0;
    int64_t total = 0;
    BatchProb* d_probs = nullptr;
    int2* d_wgmap = nullptr;
    int64_t itotal = 0;  // internal (row-padded) arena length
    float *r = nullptr, *p0 = nullptr, *p1 = nullptr;
    double* xacc = nullptr;
    double* partials = nullptr;
    unsigned* bar = nullptr;
    BatchOut* out = nullptr;
    int* err = nullptr;
    BatchOut* h_out = nullptr;  // pinned
    hipGraphExec_t graph = nullptr;
    const void* g_b = nullptr;
    const void* g_x = nullptr;
    double g_rtol2 = -1.0;
    int g_maxit = -1;
    double clock_khz = 1.0;
    std::string device_tag;
    int tuned = 0;  // problems whose tile shape was measured (not cached/given)
    int xcd_local = 0;  // problems whose barriers ran XCD-local in the last solve
    int force_agent = 0;  // 1: every group barrier takes the agent-scope fence form
    int max_restarts = BATCH_MAX_RESTARTS;  // FP64-residual restarts per problem
};

namespace {

// Resident work-groups of the persistent kernel on this device.
hipError_t batch_capacity(int* cap) {
    int dev = 0, per_cu = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_pcg, BT, 0);
    *cap = per_cu * ncu;
    return e;
}

// Every shape is legal: rows are padded to a multiple of 4 internally.
bool cfg_shape(int cfg) { return cfg == 0 || cfg == 1 || cfg == 2 || cfg == 5; }

// z-chunk for a tile shape and group size: the work-group with the most
// tiles marches ceil(tiles / G) chunks of zc planes plus ~3 planes of
// pipeline start-up each; take the zc minimising that (larger on ties).
int choose_zc(int nx, int ny, int nz, int cfg, int G) {
    const int tx = TILE_CFGS[cfg].bx * (TILE_CFGS[cfg].vec ? 4 : 1), ty = TILE_CFGS[cfg].by;
    const int64_t cross = (int64_t)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
    int best = nz;
    int64_t best_cost = INT64_MAX;
    for (int zc = nz; zc >= 1; --zc) {
        const int64_t tiles = cross * ((nz + zc - 1) / zc);
        const int64_t cost = (tiles + G - 1) / G * (zc + 3);
        if (cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
    }
    return best;
}

void set_plan(BatchProb& p, int cfg) {
    p.cfg = cfg;
    p.zc = choose_zc(p.nx, p.ny, p.nz, cfg, p.group);
    const int tx = TILE_CFGS[cfg].bx * (TILE_CFGS[cfg].vec ? 4 : 1), ty = TILE_CFGS[cfg].by;
    p.ntx = (p.nx + tx - 1) / tx;
    p.nty = (p.ny + ty - 1) / ty;
    p.nzc = (p.nz + p.zc - 1) / p.zc;
    p.ntiles = p.ntx * p.nty * p.nzc;
}

}  // namespace

// Layout and work split.
//
// Problems are packed into the arenas (each start a multiple of 64 elements,
// so 256-byte aligned for FP32 and FP64 alike). They are spread over the 8
// XCDs by longest-processing-time-first on their HBM traffic (points x
// estimated iterations), then each XCD's resident work-groups are dealt out
// greedily to the problem with the longest estimated solve time, which
// balances finish times. The estimate is a model, used only for this split,
// with constants fitted (least squares on the relative error) to the
// measured per-iteration times of the 64 problems of the uneven batch on
// MI355X:
//   iterations ~ 2.8 max(nx, ny, nz)  (Jacobi-PCG iterations grow with the
//                                      square root of the condition number)
//   one plane step of a work-group ~ 1.07 us + 1.15 ns per point of its tile
//   a phase = (busiest work-group's tiles) x (zc + 3 start-up planes) steps
//   an iteration = 2 phases + 2 x 0.45 us (the group barriers and partial
//   sums are absorbed into the per-step cost by the fit), whatever the
//   group size. (An absolute-error fit, 0.90 us + 1.11 ns and 27 us per
//   iteration, overestimates the largest problems; with the former
//   constants the batch took 54.6 ms, with these 53.8.)
namespace {

struct CostModel {
    double step0 = 1.067, step_pt = 0.00115, barrier = 0.45;
};

int model_cfg(const BatchProb& p) { return p.nx > 128 ? 2 : (p.nx > 64 ? 1 : 0); }

double model_iters(const BatchProb& p) { return 2.8 * std::max(p.nx, std::max(p.ny, p.nz)) + 1.0; }

double model_time(const BatchProb& p, int G, const CostModel& cm) {
    const int cfg = model_cfg(p);
    const int tx = TILE_CFGS[cfg].bx * (TILE_CFGS[cfg].vec ? 4 : 1), ty = TILE_CFGS[cfg].by;
    const int64_t cross = (int64_t)((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
    const double pts = (double)std::min(tx, p.nx) * std::min(ty, p.ny);
    const int zc = choose_zc(p.nx, p.ny, p.nz, cfg, G);
    const int64_t tiles = cross * ((p.nz + zc - 1) / zc);
    const double phase = (double)((tiles + G - 1) / G) * (zc + 3) * (cm.step0 + cm.step_pt * pts);
    return model_iters(p) * (2.0 * phase + 2.0 * cm.barrier);
}

}  // namespace

pcg_status batch_layout(BatchImpl& B, const int* dims, int capacity, char* msg, size_t msglen) {
    const int np = B.nprob;
    const CostModel cm;
    B.probs.assign(np, BatchProb{});
    B.cap_tiles.assign(np, 1);
    int64_t off = 0, ioff = 0;
    std::vector<double> traffic(np);
    for (int i = 0; i < np; ++i) {
        BatchProb& p = B.probs[i];
        p.nx = dims[3 * i];
        p.ny = dims[3 * i + 1];
        p.nz = dims[3 * i + 2];
        p.pitch = (p.nx + 3) / 4 * 4;
        p.off = off;
        p.ioff = ioff;
        const int64_t n = (int64_t)p.nx * p.ny * p.nz;
        off += (n + 63) / 64 * 64;
        ioff += ((int64_t)p.pitch * p.ny * p.nz + 63) / 64 * 64;
        traffic[i] = (double)n * model_iters(p);
        // most tiles any shape can give (64-point rows, 4 rows, one plane)
        B.cap_tiles[i] = (int)std::min<int64_t>(1 << 20, (int64_t)((p.nx + 63) / 64) * ((p.ny + 3) / 4) * p.nz);
    }
    B.total = off;
    B.itotal = ioff;
    const int NX = 8;
    const int per_xcd = capacity / NX;
    if (per_xcd < 1) {
        snprintf(msg, msglen, "device capacity %d is below one work-group per XCD", capacity);
        return PCG_E_UNSUPPORTED;
    }
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return traffic[a] > traffic[b]; });
    std::vector<double> load(NX, 0.0);
    std::vector<std::vector<int>> on(NX);
    for (int i : order) {
        const int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        on[best].push_back(i);
        load[best] += traffic[i];
    }
    B.wgmap.assign((size_t)per_xcd * NX, int2{-1, -1});
    B.maxg = 1;
    for (int xc = 0; xc < NX; ++xc) {
        const auto& list = on[xc];
        if (list.empty()) continue;
        if ((int)list.size() > per_xcd) {
            snprintf(msg, msglen, "%zu problems on one XCD exceed its %d resident work-groups", list.size(), per_xcd);
            return PCG_E_UNSUPPORTED;
        }
        std::vector<double> t(list.size());
        std::vector<char> full(list.size(), 0);
        for (size_t q = 0; q < list.size(); ++q) {
            B.probs[list[q]].group = 1;
            t[q] = model_time(B.probs[list[q]], 1, cm);
        }
        for (int left = per_xcd - (int)list.size(); left > 0;) {
            int w = -1;
            for (size_t q = 0; q < list.size(); ++q)
                if (!full[q] && (w < 0 || t[q] > t[w])) w = (int)q;
            if (w < 0) break;
            BatchProb& p = B.probs[list[w]];
            // (look a few work-groups ahead: the busiest work-group's tile
            // count falls in steps, so one more may not help at once)
            double ahead = t[w];
            for (int k = 1; k <= 8 && p.group + k <= B.cap_tiles[list[w]]; ++k)
                ahead = std::min(ahead, model_time(p, p.group + k, cm));
            if (ahead >= t[w]) {
                full[w] = 1;  // more work-groups would not shorten this problem
                continue;
            }
            ++p.group;
            t[w] = model_time(p, p.group, cm);
            --left;
        }
        int j = 0;
        for (int i : list) {
            BatchProb& p = B.probs[i];
            B.maxg = std::max(B.maxg, p.group);
            for (int rnk = 0; rnk < p.group; ++rnk, ++j) B.wgmap[(size_t)j * NX + xc] = int2{i, rnk};
        }
    }
    B.grid = per_xcd * NX;
    return PCG_OK;
}

}  // namespace pcgmi

using namespace pcgmi;

struct pcg_batch_s {
    BatchImpl impl;
};

namespace {

pcg_status berr(pcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(st, buf);
    return st;
}

#define BCHK(expr)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return berr(PCG_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void batch_free(BatchImpl& B) {
    if (B.graph) (void)hipGraphExecDestroy(B.graph);
    void* p[] = {B.d_probs, B.d_wgmap, B.r, B.p0, B.p1, B.xacc, B.partials, B.bar, B.out, B.err};
    for (void* q : p)
        if (q) (void)hipFree(q);
    if (B.h_out) (void)hipHostFree(B.h_out);
    if (B.capture) (void)hipStreamDestroy(B.capture);
}

// Partial slots per problem (3 buffers x 2 components x maxg), padded to
// whole 128-byte lines so no line is shared by two problems (two XCDs).
int part_stride(const BatchImpl& B) { return (6 * B.maxg + 15) / 16 * 16; }

hipError_t enqueue_batch(BatchImpl& B, const float* b, double* x, double rtol2, int maxit, hipStream_t s) {
    const int nbar = BAR_WORDS * B.nprob;
    hipLaunchKernelGGL(k_fill_u32, dim3((nbar + 255) / 256), dim3(256), 0, s, B.bar, nbar, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned*>(B.err), 1, 0u);
    hipLaunchKernelGGL(k_batch_pcg, dim3(B.grid), dim3(BT), 0, s, B.d_probs, B.d_wgmap, b, x, B.r, B.p0, B.p1,
                       B.xacc, B.partials, B.maxg, part_stride(B), B.bar, B.out, rtol2, maxit, B.err,
                       B.force_agent, B.max_restarts);
    return hipGetLastError();
}

// Upload the descriptor table; drops a captured graph (it holds old plans
// only through the table, but keep replays tied to one upload).
pcg_status upload_plans(BatchImpl& B) {
    BCHK(hipMemcpyAsync(B.d_probs, B.probs.data(), sizeof(BatchProb) * B.nprob, hipMemcpyHostToDevice, B.stream));
    BCHK(hipStreamSynchronize(B.stream));
    return PCG_OK;
}

// Run the whole batch eagerly and read back per-problem results.
pcg_status run_once(BatchImpl& B, const float* b, double* x, double rtol2, int maxit, int* herr) {
    BCHK(enqueue_batch(B, b, x, rtol2, maxit, B.stream));
    BCHK(hipMemcpyAsync(B.h_out, B.out, sizeof(BatchOut) * B.nprob, hipMemcpyDeviceToHost, B.stream));
    BCHK(hipMemcpyAsync(herr, B.err, sizeof(int), hipMemcpyDeviceToHost, B.stream));
    BCHK(hipStreamSynchronize(B.stream));
    return PCG_OK;
}

// ------------------------------------------------------------ tile cache
// One JSON object per line inside an "entries" array:
//   {"device": "gfx950:256", "nx": 16, "ny": 16, "nz": 16, "group": 3, "cfg": 2, "us": 12.5}
// keyed by device, problem shape and work-group count.
struct CacheEntry {
    std::string dev;
    int nx, ny, nz, group, cfg;
    double us;
};

std::vector<CacheEntry> cache_read(const char* path) {
    std::vector<CacheEntry> out;
    if (!path || !*path) return out;
    FILE* f = fopen(path, "r");
    if (!f) return out;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        const char* q = strstr(line, "{\"device\"");
        if (!q) continue;
        char dev[96] = {0};
        CacheEntry e{};
        if (sscanf(q, "{\"device\": \"%95[^\"]\", \"nx\": %d, \"ny\": %d, \"nz\": %d, \"group\": %d, \"cfg\": %d, \"us\": %lf",
                   dev, &e.nx, &e.ny, &e.nz, &e.group, &e.cfg, &e.us) == 7 &&
            e.cfg >= 0 && e.cfg < NUM_TILE_CFG) {
            e.dev = dev;
            out.push_back(e);
        }
    }
    fclose(f);
    return out;
}

bool cache_write(const char* path, const std::vector<CacheEntry>& es) {
    if (!path || !*path) return true;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\"format\": \"pcgmi-batch-tiles-1\", \"entries\": [\n");
    for (size_t i = 0; i < es.size(); ++i)
        fprintf(f, "  {\"device\": \"%s\", \"nx\": %d, \"ny\": %d, \"nz\": %d, \"group\": %d, \"cfg\": %d, \"us\": %.3f}%s\n",
                es[i].dev.c_str(), es[i].nx, es[i].ny, es[i].nz, es[i].group, es[i].cfg, es[i].us,
                i + 1 < es.size() ? "," : "");
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

const CacheEntry* cache_find(const std::vector<CacheEntry>& es, const std::string& dev, const BatchProb& p) {
    for (const auto& e : es)
        if (e.dev == dev && e.nx == p.nx && e.ny == p.ny && e.nz == p.nz && e.group == p.group) return &e;
    return nullptr;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Autotuner: every problem without a plan runs a fixed number of iterations
// (rtol 0) under each candidate tile shape, all problems together so that the
// measurement sees the shared HBM and L2 traffic of the real launch; each
// problem keeps the shape with the shortest wall-clock time from its start to
// its last iteration (best of `reps` launches).
pcg_status autotune(BatchImpl& B, std::vector<int>& todo, std::vector<double>& best_us, int iters, int reps) {
    Range range("batched: autotune");
    const int cands[4] = {0, 1, 2, 5};
    float* tb = nullptr;
    double* tx = nullptr;
    BCHK(hipMalloc(&tb, sizeof(float) * B.total));
    hipError_t e = hipMalloc(&tx, sizeof(double) * B.total);
    if (e != hipSuccess) {
        (void)hipFree(tb);
        return berr(PCG_E_HIP, "autotune: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, B.stream, tb, B.total, 1.0f);
    std::vector<int> best_cfg(B.nprob, -1);
    best_us.assign(B.nprob, 1e300);
    pcg_status st = PCG_OK;
    for (int c : cands) {
        for (int i : todo) set_plan(B.probs[i], c);
        if ((st = upload_plans(B)) != PCG_OK) break;
        for (int rep = 0; rep < reps && st == PCG_OK; ++rep) {
            int herr = 0;
            if ((st = run_once(B, tb, tx, 0.0, iters, &herr)) != PCG_OK) break;
            if (herr) {
                st = berr(PCG_E_HIP, "autotune: a group barrier timed out");
                break;
            }
            for (int i : todo) {
                const BatchOut& o = B.h_out[i];
                const double us = (double)(o.t_done - o.t_begin) / (B.clock_khz * 1e-3);
                if (us < best_us[i]) {
                    best_us[i] = us;
                    best_cfg[i] = B.probs[i].cfg;
                }
            }
        }
        if (st != PCG_OK) break;
    }
    (void)hipFree(tb);
    (void)hipFree(tx);
    if (st != PCG_OK) return st;
    for (int i : todo) set_plan(B.probs[i], best_cfg[i]);
    return PCG_OK;
}

}  // namespace

extern "C" {

pcg_status pcg_batch_create(pcg_batch* out, int nprob, const int* dims, const int* cfgs, const char* cache_path,
                            int tune_iters, void* hip_stream) {
    Range range("pcg_batch_create");
    if (!out || nprob < 1 || !dims) return berr(PCG_E_ARG, "pcg_batch_create: bad argument");
    *out = nullptr;
    for (int i = 0; i < nprob; ++i) {
        if (dims[3 * i] < 1 || dims[3 * i + 1] < 1 || dims[3 * i + 2] < 1)
            return berr(PCG_E_ARG, "pcg_batch_create: problem %d has a dimension < 1", i);
        if ((int64_t)dims[3 * i] * dims[3 * i + 1] * dims[3 * i + 2] > (int64_t)1 << 31)
            return berr(PCG_E_ARG, "pcg_batch_create: problem %d has more than 2^31 points", i);
        if (cfgs) {
            const int c = cfgs[i];
            if (!cfg_shape(c))
                return berr(PCG_E_ARG, "pcg_batch_create: problem %d: tile shape %d is not 0, 1, 2 or 5", i, c);
        }
    }
    if (tune_iters < 1) tune_iters = 20;
    pcg_batch bt = new (std::nothrow) pcg_batch_s();
    if (!bt) return berr(PCG_E_NOMEM, "pcg_batch_create: out of host memory");
    BatchImpl& B = bt->impl;
    B.stream = static_cast<hipStream_t>(hip_stream);
    B.nprob = nprob;
    int cap = 0, dev = 0;
    hipError_t e = batch_capacity(&cap);
    hipDeviceProp_t prop{};
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        delete bt;
        return berr(PCG_E_HIP, "pcg_batch_create: device query failed: %s", hipGetErrorString(e));
    }
    {
        char tag[160];
        snprintf(tag, sizeof tag, "%s:%d:%d", prop.gcnArchName, prop.multiProcessorCount, cap);
        for (char* c = tag; *c; ++c)
            if (*c == '"' || *c == '\\') *c = '_';
        B.device_tag = tag;
    }
    char msg[256] = {0};
    pcg_status st = batch_layout(B, dims, std::min(cap, 8192), msg, sizeof msg);
    if (st != PCG_OK) {
        delete bt;
        return berr(st, "pcg_batch_create: %s", msg);
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0) B.clock_khz = khz;
    e = hipMalloc(&B.d_probs, sizeof(BatchProb) * nprob);
    if (e == hipSuccess) e = hipMalloc(&B.d_wgmap, sizeof(int2) * B.wgmap.size());
    if (e == hipSuccess) e = hipMalloc(&B.r, sizeof(float) * B.itotal);
    if (e == hipSuccess) e = hipMalloc(&B.p0, sizeof(float) * B.itotal);
    if (e == hipSuccess) e = hipMalloc(&B.p1, sizeof(float) * B.itotal);
    if (e == hipSuccess) e = hipMalloc(&B.xacc, sizeof(double) * B.itotal);
    if (e == hipSuccess) e = hipMalloc(&B.partials, sizeof(double) * (size_t)nprob * part_stride(B));
    if (e == hipSuccess) e = hipMalloc(&B.bar, sizeof(unsigned) * BAR_WORDS * nprob);
    if (e == hipSuccess) e = hipMalloc(&B.out, sizeof(BatchOut) * nprob);
    if (e == hipSuccess) e = hipMalloc(&B.err, 64);
    if (e == hipSuccess) e = hipHostMalloc(&B.h_out, sizeof(BatchOut) * nprob, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipMemcpy(B.d_wgmap, B.wgmap.data(), sizeof(int2) * B.wgmap.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B.capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        batch_free(B);
        delete bt;
        return berr(e == hipErrorOutOfMemory ? PCG_E_NOMEM : PCG_E_HIP, "pcg_batch_create: %s", hipGetErrorString(e));
    }
    // Tile plans: given, cached, or measured.
    std::vector<int> todo;
    std::vector<CacheEntry> cache = cfgs ? std::vector<CacheEntry>{} : cache_read(cache_path);
    for (int i = 0; i < nprob; ++i) {
        BatchProb& p = B.probs[i];
        if (cfgs) {
            set_plan(p, cfgs[i]);
        } else if (const CacheEntry* ce = cache_find(cache, B.device_tag, p); ce && cfg_shape(ce->cfg)) {
            set_plan(p, ce->cfg);
        } else {
            set_plan(p, model_cfg(p));
            todo.push_back(i);
        }
    }
    if (!todo.empty()) {
        std::vector<double> us;
        st = upload_plans(B);
        if (st == PCG_OK) st = autotune(B, todo, us, tune_iters, 2);
        if (st != PCG_OK) {
            batch_free(B);
            delete bt;
            return st;
        }
        B.tuned = (int)todo.size();
        for (int i : todo) {
            const BatchProb& p = B.probs[i];
            CacheEntry ne{B.device_tag, p.nx, p.ny, p.nz, p.group, p.cfg, us[i]};
            bool found = false;
            for (auto& ce : cache)
                if (ce.dev == ne.dev && ce.nx == ne.nx && ce.ny == ne.ny && ce.nz == ne.nz && ce.group == ne.group) {
                    ce = ne;
                    found = true;
                }
            if (!found) cache.push_back(ne);
        }
        if (!cache_write(cache_path, cache)) {
            batch_free(B);
            delete bt;
            return berr(PCG_E_ARG, "pcg_batch_create: cannot write tile cache %s", cache_path);
        }
    }
    st = upload_plans(B);
    if (st != PCG_OK) {
        batch_free(B);
        delete bt;
        return st;
    }
    *out = bt;
    return PCG_OK;
}

pcg_status pcg_batch_destroy(pcg_batch bt) {
    if (!bt) return PCG_OK;
    (void)hipStreamSynchronize(bt->impl.stream);
    batch_free(bt->impl);
    delete bt;
    return PCG_OK;
}

pcg_status pcg_batch_layout(pcg_batch bt, int64_t* offsets, int64_t* total, int* plans, int* grid) {
    if (!bt) return berr(PCG_E_ARG, "pcg_batch_layout: null batch");
    const BatchImpl& B = bt->impl;
    for (int i = 0; i < B.nprob; ++i) {
        const BatchProb& p = B.probs[i];
        if (offsets) offsets[i] = p.off;
        if (plans) {
            plans[4 * i] = p.cfg;
            plans[4 * i + 1] = p.zc;
            plans[4 * i + 2] = p.group;
            plans[4 * i + 3] = p.ntiles;
        }
    }
    if (total) *total = B.total;
    if (grid) grid[0] = B.grid, grid[1] = B.tuned, grid[2] = B.xcd_local;
    return PCG_OK;
}

static int status_rank(pcg_status s) {
    return s == PCG_E_BREAKDOWN ? 3 : s == PCG_E_NOCONV ? 2 : s == PCG_E_TRUE_RESIDUAL ? 1 : 0;
}

pcg_status pcg_batch_set_barrier(pcg_batch bt, int form) {
    if (!bt) return berr(PCG_E_ARG, "pcg_batch_set_barrier: null batch");
    if (form != 0 && form != 1) return berr(PCG_E_ARG, "pcg_batch_set_barrier: form must be 0 or 1 (got %d)", form);
    BatchImpl& B = bt->impl;
    if (B.force_agent != form && B.graph) {  // the captured launch holds the old form
        BCHK(hipGraphExecDestroy(B.graph));
        B.graph = nullptr;
    }
    B.force_agent = form;
    return PCG_OK;
}

pcg_status pcg_batch_set_restarts(pcg_batch bt, int max_restarts) {
    if (!bt) return berr(PCG_E_ARG, "pcg_batch_set_restarts: null batch");
    if (max_restarts < -1) return berr(PCG_E_ARG, "pcg_batch_set_restarts: max_restarts must be >= -1");
    BatchImpl& B = bt->impl;
    const int v = max_restarts < 0 ? BATCH_MAX_RESTARTS : max_restarts;
    if (B.max_restarts != v && B.graph) {
        BCHK(hipGraphExecDestroy(B.graph));
        B.graph = nullptr;
    }
    B.max_restarts = v;
    return PCG_OK;
}

pcg_status pcg_batch_solve(pcg_batch bt, const float* b, double* x, double rtol, int maxit, int use_graph,
                           int* iters, double* relres, double* latency_s, int* restarts, double* seconds) {
    Range range("pcg_batch_solve");
    if (!bt || !b || !x) return berr(PCG_E_ARG, "pcg_batch_solve: null argument");
    if (!(rtol >= 0.0) || maxit < 0) return berr(PCG_E_ARG, "pcg_batch_solve: bad tolerance or iteration limit");
    BatchImpl& B = bt->impl;
    const auto t0 = std::chrono::steady_clock::now();
    const double rtol2 = rtol * rtol;
    if (use_graph) {
        if (!B.graph || B.g_b != b || B.g_x != x || B.g_rtol2 != rtol2 || B.g_maxit != maxit) {
            if (B.graph) {
                BCHK(hipGraphExecDestroy(B.graph));
                B.graph = nullptr;
            }
            BCHK(hipStreamBeginCapture(B.capture, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue_batch(B, b, x, rtol2, maxit, B.capture);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(B.capture, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return berr(PCG_E_HIP, "pcg_batch_solve: capture failed: %s",
                            hipGetErrorString(e != hipSuccess ? e : e2));
            }
            const hipError_t e3 = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess) {
                B.graph = nullptr;
                return berr(PCG_E_HIP, "pcg_batch_solve: instantiate failed: %s", hipGetErrorString(e3));
            }
            B.g_b = b;
            B.g_x = x;
            B.g_rtol2 = rtol2;
            B.g_maxit = maxit;
        }
        BCHK(hipGraphLaunch(B.graph, B.stream));
        BCHK(hipMemcpyAsync(B.h_out, B.out, sizeof(BatchOut) * B.nprob, hipMemcpyDeviceToHost, B.stream));
    } else {
        BCHK(enqueue_batch(B, b, x, rtol2, maxit, B.stream));
        BCHK(hipMemcpyAsync(B.h_out, B.out, sizeof(BatchOut) * B.nprob, hipMemcpyDeviceToHost, B.stream));
    }
    int herr = 0;
    BCHK(hipMemcpyAsync(&herr, B.err, sizeof(int), hipMemcpyDeviceToHost, B.stream));
    BCHK(hipStreamSynchronize(B.stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (seconds) *seconds = secs;
    if (herr) return berr(PCG_E_HIP, "pcg_batch_solve: a group barrier timed out (work-groups not co-resident)");
    unsigned long long tmin = ~0ull;
    B.xcd_local = 0;
    for (int i = 0; i < B.nprob; ++i) {
        tmin = std::min(tmin, B.h_out[i].t_begin);
        B.xcd_local += B.h_out[i].xcd_local;
    }
    pcg_status ret = PCG_OK;
    for (int i = 0; i < B.nprob; ++i) {
        const BatchOut& o = B.h_out[i];
        if (iters) iters[i] = o.iters;
        if (relres) relres[i] = o.rr0 > 0 ? std::sqrt(o.rr_true / o.rr0) : 0.0;
        if (restarts) restarts[i] = o.restarts;
        if (latency_s) latency_s[i] = (double)(o.t_done - tmin) / (B.clock_khz * 1e3);
        // worst outcome over the problems: breakdown, then maxit, then a
        // converged recursion whose FP64 true residual is above rtol
        const pcg_status pst = o.done == 2 ? PCG_E_BREAKDOWN
                               : o.done != 1 ? PCG_E_NOCONV
                               : !(o.rr_true <= rtol2 * o.rr0) ? PCG_E_TRUE_RESIDUAL : PCG_OK;
        if (status_rank(pst) > status_rank(ret)) ret = pst;
    }
    if (ret == PCG_E_TRUE_RESIDUAL)
        berr(ret, "pcg_batch_solve: some problems stopped with an FP64 true residual above rtol");
    else if (ret != PCG_OK) berr(ret, "pcg_batch_solve: some problems did not converge");
    return ret;
}

}  // extern "C"
