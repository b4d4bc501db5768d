// runtime.hip -- the C ABI (include/pcgmi.h): contexts, workspace, argument
// checking, error reporting and the PCG driver loop.
//
// The driver keeps every scalar of the iteration on the device (paper Sec. VII
// keeps the BF16 solver's residual norm on the device for the same reason:
// no host round trip per iteration). Iterations are replayed as captured HIP
// graph chunks of C iterations; after each chunk a 96-byte copy of the solve
// state goes to pinned host memory. The host waits on the PREVIOUS chunk's
// copy while the current one runs, so the GPU never idles on the check; the
// kernels of a chunk that starts after convergence return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "ops.hpp"
#include "pcgmi.h"
#include "trace.hpp"

using namespace pcgmi;

namespace {

thread_local std::string g_err;

pcg_status fail(pcg_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pcg_status fail(pcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(PCG_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Do [a, a + abytes) and [b, b + bbytes) intersect?
bool overlap2(const void* a, size_t abytes, const void* b, size_t bbytes) {
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return abytes > 0 && bbytes > 0 && x < y + bbytes && y < x + abytes;
}

bool overlap(const void* a, const void* b, size_t bytes) { return overlap2(a, bytes, b, bytes); }

}  // namespace

namespace pcgmi {

// Record an error message for pcg_last_error() from other translation units.
const char* set_error(pcg_status st, const char* msg) {
    (void)st;
    g_err = msg;
    return g_err.c_str();
}

Geometry make_geometry(int nx, int ny, int nz, const Plan& p, int dt) {
    Geometry g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    const int tx = plan_tx(p, dt), ty = plan_ty(p);
    g.ntx = (nx + tx - 1) / tx;
    g.nty = (ny + ty - 1) / ty;
    g.zc = std::max(1, std::min(p.zc, nz));
    g.nzc = (nz + g.zc - 1) / g.zc;
    g.nblocks = (unsigned)g.ntx * (unsigned)g.nty * (unsigned)g.nzc;
    g.pitch = nx;
    return g;
}

}  // namespace pcgmi

struct pcg_ctx_s {
    int nx = 0, ny = 0, nz = 0;
    int64_t n = 0;
    int dt = DT_F32;
    hipStream_t stream = nullptr;   // caller's stream
    hipStream_t capture = nullptr;  // private stream used only to capture graphs
    pcg_options opt{};
    Plan plan{};
    Geometry geo{};      // iteration kernels (the direction kernel's)
    Plan plan_upd{};
    Geometry geo_upd{};  // the update kernel's (a taller z-chunk by default)
    Plan plan_res{};
    Geometry geo_res{};  // FP64 residual kernel
    // workspace
    void* r = nullptr;
    void* p[2] = {nullptr, nullptr};
    void* xacc = nullptr;  // x accumulator, type opt.x_accum
    double* partials = nullptr;
    size_t partials_cap = 0;  // doubles
    unsigned* ticket = nullptr;
    SolveState* st = nullptr;
    double* hist = nullptr;
    int hist_cap = 0;
    double* res2 = nullptr;  // {||r||^2, max|r|}
    // pinned host mirrors
    SolveState* hst = nullptr;  // [2] ping-pong copies of the device state
    double* hres = nullptr;     // [2]
    // graph chunk
    hipGraphExec_t chunk = nullptr;
    bool chunk_sr = false;  // the captured chunk holds single-reduction iterations
    int chunk_iters = 0;
    // single-reduction form: r (second), w (two), s (two) in one allocation
    void* sr = nullptr;
    bool sr_active = false;
    hipEvent_t ev_chunk[2] = {nullptr, nullptr};
    int last_iters = 0;
    // operator: constant coefficients unless pcg_set_coefficients gave k
    const float* kc = nullptr;  // caller's cell coefficients (device, FP32)
    void* dinv = nullptr;       // inverse Jacobi diagonal (storage type), owned
    // flexible CG
    void* q = nullptr;  // A p (storage type)
    void* z = nullptr;  // preconditioned residual (storage type)
    // captured flexible iterations: [0] Jacobi, [1] with the network, [2]
    // with the multigrid V-cycle, and what they were recorded with
    hipGraphExec_t flex_exec[3] = {nullptr, nullptr, nullptr};
    struct FlexKey {
        cnn_net net = nullptr;
        const float* g = nullptr;
        uint64_t epoch = 0;
        const void* hist = nullptr;
        const float* kc = nullptr;
        int chunk = 0;
        uint64_t mg_epoch = 0;
    } flex_key[3];
    // multigrid hierarchy (pcg_set_multigrid) and the memory it owns
    MgHierarchy* mg = nullptr;
    std::vector<void*> mg_mem;
    int mg_nu = 1, mg_coarse_max = 512;
    double mg_omega = 6.0 / 7.0;
    uint64_t mg_epoch = 0;   // bumped on every rebuild (captured graphs hold its pointers)
    int* zero_flag = nullptr;  // a device int kept at 0 (the V-cycle's "done" outside a solve)
    // iterative refinement
    void* rhat = nullptr;  // scaled residual in the storage type
    std::vector<double> ref_relres;
    std::vector<int> ref_inner;
};

namespace {

Red red_of(pcg_ctx c) { return Red{c->partials, c->ticket, c->partials_cap}; }
OpDesc op_of(pcg_ctx c) { return OpDesc{c->kc, c->kc ? c->dinv : nullptr}; }

}  // namespace

// Access for the network's A-norm loss (same library): the context's
// operator on FP32 vectors, its Jacobi scale, dims and stream.
namespace pcgmi {
hipError_t ctx_apply_f32(pcg_ctx c, const float* u, float* y) {
    return launch_stencil(DT_F32, c->plan, c->geo, op_of(c), u, y, c->stream);
}
const float* ctx_dinv_f32(pcg_ctx c) { return static_cast<const float*>(op_of(c).dinv); }
bool ctx_is_f32_grid(pcg_ctx c, int nx, int ny, int nz) {
    return c->dt == DT_F32 && c->nx == nx && c->ny == ny && c->nz == nz;
}
hipStream_t ctx_stream(pcg_ctx c) { return c->stream; }
}  // namespace pcgmi

namespace {

void free_ctx(pcg_ctx c) {
    if (!c) return;
    if (c->chunk) (void)hipGraphExecDestroy(c->chunk);
    for (auto& fe : c->flex_exec)
        if (fe) (void)hipGraphExecDestroy(fe);
    for (auto& e : c->ev_chunk)
        if (e) (void)hipEventDestroy(e);
    void* dev[] = {c->r, c->p[0], c->p[1], c->xacc, c->partials, c->ticket, c->st, c->hist, c->res2, c->rhat,
                   c->dinv, c->q, c->z, c->sr};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    if (c->hst) (void)hipHostFree(c->hst);
    if (c->hres) (void)hipHostFree(c->hres);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    for (void* d : c->mg_mem)
        if (d) (void)hipFree(d);
    if (c->zero_flag) (void)hipFree(c->zero_flag);
    delete c->mg;
    delete c;
}

// Default plan (measured on MI355X with the split reductions): when the x-y
// plane is small (<= 65536 points, e.g. 256^3) FP32 128 x 8 and FP64 128 x 4
// footprints with 32-plane chunks, 16-bit 256 x 8 with 16-plane chunks; on
// larger planes 256 x 4 FP32 / 512 x 4 16-bit / 128 x 4 FP64 footprints
// with 16-plane chunks (8 for 16-bit); chunks halved while the launch has
// fewer than 256 work-groups; the scalar shape when nx is not a multiple of
// the 16-byte vector width. 16-bit sweeps: the BF16 refinement's inner
// iteration at 256^3 ran at 5.15 TB/s with 256 x 8 / 16 planes against 4.86
// with 128 x 16 / 8 planes (18 plans, 4.04-5.15); the 512^3 BF16 stencil took
// 77.5 us with 512 x 4 / 8 planes against 85.1 with 128 x 16 / 16.
Plan default_plan(int nx, int ny, int nz, int dt, const pcg_options& o) {
    const bool small_plane = (int64_t)nx * ny <= 65536;
    const int w = dt_width(dt);  // 4 FP32, 8 16-bit, 2 FP64
    Plan p{2, small_plane ? (w == 8 ? 16 : 32) : (w == 8 ? 8 : 16)};
    if (w == 8 && small_plane) p.cfg = 1;        // 32 x 8 threads: 256 x 8 points
    else if (w == 4 && small_plane) p.cfg = 1;   // 32 x 8 threads: 128 x 8 points
    // narrower vector shapes while the footprint is wider than nx
    if (plan_tx(p, dt) > nx && p.cfg == 2) p.cfg = 1;
    if (plan_tx(p, dt) > nx && p.cfg == 1) p.cfg = 0;
    if (nx % w != 0) p.cfg = 5;
    if (o.tile_x > 0 || o.tile_y > 0) {
        for (int c = 0; c < NUM_TILE_CFG; ++c) {
            Plan q{c, 1};
            if ((o.tile_x <= 0 || plan_tx(q, dt) == o.tile_x) && (o.tile_y <= 0 || plan_ty(q) == o.tile_y) &&
                (TILE_CFGS[c].vec == (p.cfg != 5))) {
                p.cfg = c;
                break;
            }
        }
    }
    const int64_t tiles = (int64_t)((nx + plan_tx(p, dt) - 1) / plan_tx(p, dt)) *
                          ((ny + plan_ty(p) - 1) / plan_ty(p));
    int64_t zc = p.zc;
    // keep at least ~256 work-groups when the grid allows it
    while (zc > 4 && tiles * ((nz + zc - 1) / zc) < 256) zc /= 2;
    p.zc = o.zchunk > 0 ? o.zchunk : (int)zc;
    return p;
}

pcg_status ensure_hist(pcg_ctx c, int maxit) {
    if (maxit + 1 <= c->hist_cap) return PCG_OK;
    if (c->hist) HIPCHK(hipFree(c->hist));
    c->hist = nullptr;
    int cap = std::max(maxit + 1, 1024);
    HIPCHK(hipMalloc(&c->hist, sizeof(double) * cap));
    c->hist_cap = cap;
    if (c->chunk) {  // captured kernels hold the old pointer
        HIPCHK(hipGraphExecDestroy(c->chunk));
        c->chunk = nullptr;
    }
    return PCG_OK;
}

// Enqueue iterations [first, first + count) on stream s. Iteration i reads
// the direction buffer p[(i - 1) & 1] and writes p[i & 1]. The kernels chain
// their reductions: the state the host reads (st[0]) is current before the
// first direction kernel and after the closing kernel; in between, each
// update kernel writes st[1] from st[0] and each later direction kernel st[0]
// from st[1]. Direction partials go to the first half of the partials
// buffer, update partials (two components at most) to the second.
// Single-reduction iterations [first, first + count) (count even). Global
// iteration k = i - 1 reads r[k & 1], w[k & 1], s[(k + 1) & 1] and writes
// the other buffer of each (halo points of the inputs are read while
// neighbouring work-groups write their outputs); p and x are updated in
// place (own points only). The kernels chain their reductions over the two
// state buffers as the two-kernel form does, so st[0] is current again after
// the closing kernel.
hipError_t enqueue_iters_sr(pcg_ctx c, int first, int count, hipStream_t s, hipEvent_t* evs) {
    if (count <= 0) return hipSuccess;
    if (count & 1) return hipErrorInvalidValue;
    const size_t vb = (size_t)c->n * dt_size(c->dt);
    char* base = static_cast<char*>(c->sr);
    void* R[2] = {c->r, base};
    void* W[2] = {base + vb, base + 2 * vb};
    void* S[2] = {base + 3 * vb, base + 4 * vb};
    SolveState* st[2] = {c->st, c->st + 1};
    double* part[2] = {c->partials, c->partials + c->partials_cap / 2};
    const unsigned nb = c->geo.nblocks;
    for (int i = first; i < first + count; ++i) {
        const int k = i - 1, j = i - first;
        const SRBufs bufs{R[k & 1], W[k & 1], S[(k + 1) & 1], R[(k + 1) & 1], W[(k + 1) & 1], S[k & 1], c->p[0]};
        const Chain ch = j == 0 ? Chain{nullptr, nb, st[0], st[0], c->hist, part[0]}
                                : Chain{part[(j - 1) & 1], nb, st[(j + 1) & 1], st[j & 1], c->hist, part[j & 1]};
        if (evs) (void)hipEventRecord(evs[3 * j], s);
        hipError_t e = launch_pcg_sr(c->dt, c->plan, c->geo, bufs, c->xacc, c->opt.x_accum, ch, s);
        if (e != hipSuccess) return e;
        if (evs) {
            (void)hipEventRecord(evs[3 * j + 1], s);
            (void)hipEventRecord(evs[3 * j + 2], s);
        }
    }
    return launch_pcg_sr_close(Chain{part[(count - 1) & 1], nb, st[(count + 1) & 1], st[count & 1], c->hist, nullptr}, s);
}

// Iterations first .. first + count - 1 of the two-kernel form. x advances
// every second iteration (x_defer; odd iterations leave it, even ones add
// both steps); every_x, or x_defer = 0: every iteration leaves x current
// (the update skips x and k_x_finish adds alpha p from the update's state).
hipError_t enqueue_iters(pcg_ctx c, int first, int count, hipStream_t s, hipEvent_t* evs, bool every_x = false) {
    if (c->sr_active) return enqueue_iters_sr(c, first, count, s, evs);
    if (count <= 0) return hipSuccess;
    SolveState* s0 = c->st;
    SolveState* s1 = c->st + 1;
    double* pdir = c->partials;
    double* pupd = c->partials + c->partials_cap / 2;
    const unsigned nbd = c->geo.nblocks;
    const bool defer = c->opt.x_defer && !every_x;
    unsigned nlast = c->geo_upd.nblocks;  // partials left by the previous update
    for (int i = first; i < first + count; ++i) {
        void* pold = c->p[(i - 1) & 1];
        void* pnew = c->p[i & 1];
        if (evs) (void)hipEventRecord(evs[3 * (i - first)], s);
        const Chain dch =
            i == first ? Chain{nullptr, nlast, s0, s0, c->hist, pdir} : Chain{pupd, nlast, s1, s0, c->hist, pdir};
        hipError_t e = launch_pcg_direction(c->dt, c->plan, c->geo, op_of(c), c->r, pold, pnew, dch, s);
        if (e != hipSuccess) return e;
        if (evs) (void)hipEventRecord(evs[3 * (i - first) + 1], s);
        const Chain uch{pdir, nbd, s0, s1, c->hist, pupd};
        // An update that adds to x streams the most bytes and takes the
        // update plan; one that leaves x moves what the direction kernel
        // moves and takes its plan.
        const int xmode = defer && (i & 1) == 0 ? 2 : 1;
        const Plan& up = xmode == 2 ? c->plan_upd : c->plan;
        const Geometry& ug = xmode == 2 ? c->geo_upd : c->geo;
        e = launch_pcg_update(c->dt, up, ug, op_of(c), pnew, c->xacc, c->opt.x_accum, c->r, xmode, pold, uch, s);
        if (e != hipSuccess) return e;
        nlast = ug.nblocks;
        if (!defer) {
            e = launch_x_finish(c->dt, c->opt.x_accum, c->n, c->xacc, pnew, s1, true, s);
            if (e != hipSuccess) return e;
        }
        if (evs) (void)hipEventRecord(evs[3 * (i - first) + 2], s);
    }
    return launch_pcg_close(op_of(c).kc != nullptr, Chain{pupd, nlast, s1, s0, c->hist, nullptr}, s);
}

pcg_status ensure_chunk(pcg_ctx c) {
    if (c->chunk && c->chunk_sr != c->sr_active) {
        HIPCHK(hipGraphExecDestroy(c->chunk));
        c->chunk = nullptr;
    }
    if (c->chunk) return PCG_OK;
    Range range("graph capture: PCG iterations");
    c->chunk_sr = c->sr_active;
    if (!c->capture) HIPCHK(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_iters(c, 1, c->chunk_iters, c->capture, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->capture, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(PCG_E_HIP, "capturing the iteration chunk failed: %s", hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(PCG_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(&c->chunk, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) {
        c->chunk = nullptr;
        return fail(PCG_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
    }
    return PCG_OK;
}


struct IterResult {
    SolveState fin{};
    double k1_ms = 0.0, k2_ms = 0.0;
    int nk = 0;
    double k2e_ms = 0.0;  // the updates of even iterations (those that advance x)
    int nke = 0;
};

// Single-reduction iterations (constant coefficients only): forced by the
// option, or chosen by size when it is -1. Measured per iteration on MI355X
// (FP32 storage, FP64 x): 64^3 12.5 us against 14.8 us for two kernels,
// 128^3 equal, 512 x 112 x 64 37.1 against 33.1, 256^3 174 against 113 (the
// fused kernel moves 48 B/pt and stages three halo streams). Its recursive
// residual also drifts further from b - A x (the recurrence for s = A p adds
// rounding): with b = A x* for a smooth x* the FP64 judge restarts it later,
// and whole solves to a true 1e-6 measured 32^3 1.23 against 1.38 ms, 48^3
// 1.83 against 1.86, 64^3 2.43 against 2.21. With 16-bit storage it takes
// more iterations. So: FP32/FP64 storage up to 2^17 points (about 50^3).
bool want_single_reduction(pcg_ctx c) {
    if (c->kc != nullptr) return false;
    if (c->opt.single_reduction >= 0) return c->opt.single_reduction != 0;
    return (c->dt == DT_F32 || c->dt == DT_F64) && c->n <= ((int64_t)1 << 17);
}

// Start a solve of A x = b on the workspace (x0 = 0, or x0 given in x0 of
// type x0_dt) and run PCG iterations until the device state says done:
// converged, breakdown, maxit, or (stag > 0) no 10% improvement of the best
// residual for stag iterations. The iterate is left in c->xacc.
pcg_status run_iterations(pcg_ctx c, const void* b, const void* x0, int x0_dt, double rtol, int maxit, int stag,
                          IterResult* out) {
    pcg_status s = ensure_hist(c, maxit);
    if (s != PCG_OK) return s;
    hipStream_t st = c->stream;
    const int xacc_dt = c->opt.x_accum;

    // Host-side initial state: rtol^2 (scaled by ||b||^2 on the device), 1/6, maxit.
    SolveState init{};
    init.tol2 = rtol * rtol;
    init.dinv = 1.0 / 6.0;
    init.maxit = maxit;
    init.stag = stag;
    c->hst[0] = init;
    HIPCHK(hipMemcpyAsync(c->st, &c->hst[0], sizeof(SolveState), hipMemcpyHostToDevice, st));
    if (x0) {
        if (x0 != c->xacc) HIPCHK(launch_convert(x0_dt, xacc_dt, c->n, x0, c->xacc, st));
        HIPCHK(launch_zero(c->dt, c->n, c->p[0], st));
        HIPCHK(launch_zero(c->dt, c->n, c->p[1], st));
        HIPCHK(launch_pcg_start_x0(c->dt, xacc_dt, c->plan_res, c->geo_res, op_of(c), b, c->xacc, c->r, c->st,
                                   c->hist, red_of(c), st));
    } else {
        HIPCHK(launch_pcg_start_zero(c->dt, c->n, b, c->r, c->xacc, xacc_dt, c->p[0], op_of(c).dinv, c->st,
                                     c->hist, red_of(c), st));
    }
    c->sr_active = want_single_reduction(c);
    if (c->sr_active) {
        // w0 = A D^-1 r0 and {gamma0, delta0}; s_{-1} = 0 (p_{-1} = 0 from the start above)
        const size_t vb = (size_t)c->n * dt_size(c->dt);
        if (!c->sr) HIPCHK(hipMalloc(&c->sr, 5 * vb));
        char* base = static_cast<char*>(c->sr);
        HIPCHK(launch_zero(c->dt, c->n, base + 4 * vb, st));
        HIPCHK(launch_pcg_sr_start(c->dt, c->plan, c->geo, c->r, base + vb, c->st, red_of(c), st));
    }

    const int C = c->chunk_iters;
    const bool timing = c->opt.kernel_timing != 0;
    const bool graph = c->opt.use_graph && !timing;
    if (graph) {
        s = ensure_chunk(c);
        if (s != PCG_OK) return s;
    }
    hipEvent_t* evs = nullptr;
    std::vector<float> k1_each, k2_each;  // per-iteration kernel times (timing mode)
    if (timing) {
        evs = new hipEvent_t[3 * C];
        for (int i = 0; i < 3 * C; ++i) (void)hipEventCreate(&evs[i]);
    }
    struct EvGuard {
        hipEvent_t*& e;
        int n;
        ~EvGuard() {
            if (e) {
                for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
                delete[] e;
                e = nullptr;
            }
        }
    } guard{evs, 3 * C};

    // Chunk loop: launch chunk k, queue its state copy, then wait for chunk k-1's copy.
    int launched = 0, slot = 0;
    bool finished = false;
    SolveState& fin = out->fin;
    HIPCHK(hipMemcpyAsync(&c->hst[1], c->st, sizeof(SolveState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(c->ev_chunk[1], st));
    HIPCHK(hipEventSynchronize(c->ev_chunk[1]));
    fin = c->hst[1];
    if (fin.done != 0) finished = true;
    bool pending = false;
    int pend_slot = 0;
    while (!finished) {
        if (launched < maxit) {
            hipError_t e;
            if (graph) e = hipGraphLaunch(c->chunk, st);
            else e = enqueue_iters(c, launched + 1, C, st, evs);
            if (e != hipSuccess) return fail(PCG_E_HIP, "launching PCG iterations failed: %s", hipGetErrorString(e));
            launched += C;
            if (timing) {
                // Eager timing mode: wait for this chunk and sum its kernel times.
                (void)hipEventSynchronize(evs[3 * C - 1]);
                for (int i = 0; i < C; ++i) {
                    float a = 0.f, b2 = 0.f;
                    (void)hipEventElapsedTime(&a, evs[3 * i], evs[3 * i + 1]);
                    (void)hipEventElapsedTime(&b2, evs[3 * i + 1], evs[3 * i + 2]);
                    k1_each.push_back(a);
                    k2_each.push_back(b2);
                }
            }
            HIPCHK(hipMemcpyAsync(&c->hst[slot], c->st, sizeof(SolveState), hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(c->ev_chunk[slot], st));
        }
        if (pending) {
            HIPCHK(hipEventSynchronize(c->ev_chunk[pend_slot]));
            fin = c->hst[pend_slot];
            if (fin.done != 0) finished = true;
        }
        if (launched >= maxit && !finished) {
            // Nothing more to launch: wait for the last chunk.
            HIPCHK(hipEventSynchronize(c->ev_chunk[slot]));
            fin = c->hst[slot];
            finished = true;
        }
        pending = true;
        pend_slot = slot;
        slot ^= 1;
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(&fin, c->st, sizeof(SolveState), hipMemcpyDeviceToHost));
    c->last_iters = fin.iters;
    // x advances every second iteration: after an odd count it still owes
    // the last step (its direction is in p[1], its alpha in the state).
    if (!c->sr_active && c->opt.x_defer && (fin.iters & 1)) {
        HIPCHK(launch_x_finish(c->dt, c->opt.x_accum, c->n, c->xacc, c->p[1], c->st, false, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    // Only iterations that did work count (later launches of the last chunk
    // return at once).
    const int nwork = std::min<int>(fin.iters, (int)k1_each.size());
    for (int i = 0; i < nwork; ++i) {
        out->k1_ms += k1_each[i];
        out->k2_ms += k2_each[i];
        if ((i & 1) == 1) {  // iteration i + 1 is even
            out->k2e_ms += k2_each[i];
            ++out->nke;
        }
    }
    out->nk = nwork;
    return PCG_OK;
}

}  // namespace

namespace {

// Dense seven-point operator of an nx x ny x nz grid in FP64 (row-major):
// face coefficients 1 (kcell empty) or the harmonic mean of the two cells'
// k, a boundary face taking its cell's k (the operator the z-march kernels
// apply with StencilConst / StencilVar).
std::vector<double> dense_operator(int nx, int ny, int nz, const std::vector<float>& kcell) {
    const int m = nx * ny * nz;
    std::vector<double> A((size_t)m * m, 0.0);
    auto idx = [&](int i, int j, int k) { return (k * ny + j) * nx + i; };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int p = idx(i, j, k);
                const double kp = kcell.empty() ? 1.0 : (double)kcell[p];
                double diag = 0.0;
                const int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
                for (const auto& q : nb) {
                    const bool in = q[0] >= 0 && q[0] < nx && q[1] >= 0 && q[1] < ny && q[2] >= 0 && q[2] < nz;
                    double kf = kp;
                    if (in && !kcell.empty()) {
                        const double kq = (double)kcell[idx(q[0], q[1], q[2])];
                        kf = 2.0 * kp * kq / (kp + kq);
                    }
                    diag += kf;
                    if (in) A[(size_t)p * m + idx(q[0], q[1], q[2])] -= kf;
                }
                A[(size_t)p * m + p] = diag;
            }
    return A;
}

// Inverse of a symmetric positive definite matrix (row-major, m x m) through
// its Cholesky factor A = L L^T: Y = L^-1 (lower triangular, row i from rows
// 0..i-1 of Y), then A^-1 = Y^T Y, summed as outer products of Y's rows. Every
// inner loop runs along a row, so the m^3 work streams through memory.
// False if a pivot is not positive.
bool spd_inverse(const std::vector<double>& A, int m, std::vector<double>& inv) {
    const size_t M = (size_t)m;
    std::vector<double> L(M * M, 0.0);
    for (int j = 0; j < m; ++j) {
        const double* lj = &L[j * M];
        double d = A[j * M + j];
        for (int k = 0; k < j; ++k) d -= lj[k] * lj[k];
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L[j * M + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            const double* li = &L[i * M];
            double t = A[i * M + j];
            for (int k = 0; k < j; ++k) t -= li[k] * lj[k];
            L[i * M + j] = t / ljj;
        }
    }
    // Y = L^-1: Y[i][0..i] = (e_i - sum_{k<i} L[i][k] Y[k][0..k]) / L[i][i]
    std::vector<double> Y(M * M, 0.0);
    for (int i = 0; i < m; ++i) {
        double* yi = &Y[i * M];
        yi[i] = 1.0;
        for (int k = 0; k < i; ++k) {
            const double lik = L[i * M + k];
            const double* yk = &Y[k * M];
            for (int c = 0; c <= k; ++c) yi[c] -= lik * yk[c];
        }
        const double r = 1.0 / L[i * M + i];
        for (int c = 0; c <= i; ++c) yi[c] *= r;
    }
    // A^-1 = Y^T Y: lower triangle from the rows' outer products, then mirrored
    inv.assign(M * M, 0.0);
    for (int i = 0; i < m; ++i) {
        const double* yi = &Y[i * M];
        for (int a = 0; a <= i; ++a) {
            const double ya = yi[a];
            double* row = &inv[(size_t)a * M];
            for (int b = 0; b <= a; ++b) row[b] += ya * yi[b];
        }
    }
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < a; ++b) inv[(size_t)b * M + a] = inv[(size_t)a * M + b];
    return true;
}

constexpr int MG_COARSEST_MAX = 1024;  // points of the coarsest grid (dense inverse)

void free_mg(pcg_ctx c) {
    for (void* d : c->mg_mem)
        if (d) (void)hipFree(d);
    c->mg_mem.clear();
    delete c->mg;
    c->mg = nullptr;
    if (c->flex_exec[2]) {
        (void)hipGraphExecDestroy(c->flex_exec[2]);
        c->flex_exec[2] = nullptr;
    }
}

// Builds the hierarchy for the context's current operator.
pcg_status build_mg(pcg_ctx c) {
    Range range("multigrid setup");
    hipStream_t st = c->stream;
    HIPCHK(hipStreamSynchronize(st));
    free_mg(c);
    auto alloc = [&](size_t bytes, void** out) -> hipError_t {
        hipError_t e = hipMalloc(out, bytes);
        if (e == hipSuccess) c->mg_mem.push_back(*out);
        return e;
    };
    if (!c->zero_flag) {
        HIPCHK(hipMalloc(&c->zero_flag, sizeof(int)));
        HIPCHK(hipMemsetAsync(c->zero_flag, 0, sizeof(int), st));
    }
    MgHierarchy* H = new (std::nothrow) MgHierarchy();
    if (!H) return fail(PCG_E_NOMEM, "pcg_set_multigrid: out of host memory");
    c->mg = H;
    H->nu = c->mg_nu;
    H->omega = (float)c->mg_omega;
    pcg_options dflt;
    pcg_options_default(&dflt);
    int nx = c->nx, ny = c->ny, nz = c->nz;
    for (int l = 0; l < MG_MAX_LEVELS; ++l) {
        MgLevel& L = H->lv[l];
        L.nx = nx;
        L.ny = ny;
        L.nz = nz;
        L.n = (int64_t)nx * ny * nz;
        L.plan = default_plan(nx, ny, nz, DT_F32, l == 0 ? c->opt : dflt);
        L.geo = make_geometry(nx, ny, nz, L.plan, DT_F32);
        H->nlev = l + 1;
        if (L.n <= c->mg_coarse_max || nx % 2 || ny % 2 || nz % 2 || l + 1 == MG_MAX_LEVELS) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
    }
    const int last = H->nlev - 1;
    if (H->lv[last].n > MG_COARSEST_MAX) {
        free_mg(c);
        return fail(PCG_E_UNSUPPORTED,
                    "pcg_set_multigrid: the coarsest grid (%dx%dx%d) has more than %d points; every dimension must "
                    "halve evenly down to at most that many",
                    H->lv[last].nx, H->lv[last].ny, H->lv[last].nz, MG_COARSEST_MAX);
    }
    const bool var = c->kc != nullptr;
    for (int l = 0; l <= last; ++l) {
        MgLevel& L = H->lv[l];
        const size_t b = sizeof(float) * (size_t)L.n;
        void* t = nullptr;
        if (l > 0) {
            HIPCHK(alloc(b, &t));
            L.g = static_cast<float*>(t);
            HIPCHK(alloc(b, &t));
            L.out = static_cast<float*>(t);
        }
        if (l < last) {
            HIPCHK(alloc(b, &t));
            L.u[0] = static_cast<float*>(t);
            if (H->nu >= 2) {
                HIPCHK(alloc(b, &t));
                L.u[1] = static_cast<float*>(t);
            }
            HIPCHK(alloc(b, &t));
            L.r = static_cast<float*>(t);
        }
        if (var) {
            if (l == 0) {
                L.k = c->kc;
                L.dinv = static_cast<const float*>(c->dinv);
            } else {
                const MgLevel& F = H->lv[l - 1];
                HIPCHK(alloc(b, &t));
                HIPCHK(launch_mg_coarsen_k(F.k, F.nx, F.ny, F.nz, static_cast<float*>(t), st));
                L.k = static_cast<float*>(t);
                HIPCHK(alloc(b, &t));
                HIPCHK(launch_var_dinv(DT_F32, L.plan, L.geo, L.k, t, st));
                L.dinv = static_cast<float*>(t);
            }
        }
    }
    // coarsest operator, inverted on the host in FP64
    const MgLevel& C = H->lv[last];
    const int m = (int)C.n;
    std::vector<float> kh;
    if (var) {
        kh.resize(m);
        HIPCHK(hipMemcpyAsync(kh.data(), C.k, sizeof(float) * m, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    std::vector<double> inv;
    if (!spd_inverse(dense_operator(C.nx, C.ny, C.nz, kh), m, inv)) {
        free_mg(c);
        return fail(PCG_E_ARG, "pcg_set_multigrid: the coarsest operator is not positive definite (k <= 0?)");
    }
    std::vector<float> inv32(inv.begin(), inv.end());
    void* t = nullptr;
    HIPCHK(alloc(sizeof(float) * inv32.size(), &t));
    H->ainv = static_cast<float*>(t);
    HIPCHK(hipMemcpyAsync(H->ainv, inv32.data(), sizeof(float) * inv32.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    ++c->mg_epoch;
    return PCG_OK;
}

}  // namespace

extern "C" {

const char* pcg_last_error(void) { return g_err.c_str(); }

pcg_status pcg_options_default(pcg_options* o) {
    if (!o) return fail(PCG_E_ARG, "pcg_options_default: null options");
    std::memset(o, 0, sizeof *o);
    o->chunk_iters = 16;
    o->x_accum = -1;  // resolved at pcg_create: FP64
    o->x_dtype = -1;  // resolved at pcg_create: F32 storage -> F32, otherwise storage type
    o->use_graph = 1;
    o->stag_window = -1;
    o->max_restarts = -1;
    o->single_reduction = -1;
    o->x_defer = 1;
    return PCG_OK;
}

pcg_status pcg_create(pcg_ctx* out, int nx, int ny, int nz, pcg_dtype storage, void* hip_stream,
                      const pcg_options* opt) {
    if (!out) return fail(PCG_E_ARG, "pcg_create: null output handle");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(PCG_E_ARG, "pcg_create: dims must be >= 1 (got %d %d %d)", nx, ny, nz);
    const int64_t n = (int64_t)nx * ny * nz;
    if (n > (int64_t(1) << 33)) return fail(PCG_E_ARG, "pcg_create: grid too large (%lld points)", (long long)n);
    if (storage < PCG_F32 || storage > PCG_F64) return fail(PCG_E_ARG, "pcg_create: bad storage dtype %d", (int)storage);
    pcg_options o;
    pcg_options_default(&o);
    if (opt) o = *opt;
    o.x_defer = o.x_defer != 0;
    if (o.chunk_iters <= 0) o.chunk_iters = 16;
    if (o.chunk_iters & 1) ++o.chunk_iters;
    if (o.x_dtype < 0) o.x_dtype = storage;
    if (o.x_dtype != storage && o.x_dtype != PCG_F64)
        return fail(PCG_E_ARG, "pcg_create: x_dtype must be the storage type or PCG_F64");
    if (o.x_accum < 0) o.x_accum = PCG_F64;
    if (o.stag_window < 0) o.stag_window = 100;
    if (o.max_restarts < 0) o.max_restarts = 3;
    if (o.x_accum != PCG_F64 && o.x_accum != PCG_F32 && o.x_accum != storage)
        return fail(PCG_E_ARG, "pcg_create: x_accum must be PCG_F64, PCG_F32 or the storage type");
    if (storage == PCG_F64) o.x_accum = PCG_F64;

    pcg_ctx c = new (std::nothrow) pcg_ctx_s();
    if (!c) return fail(PCG_E_NOMEM, "pcg_create: out of host memory");
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->n = n;
    c->dt = storage;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->opt = o;
    c->plan = default_plan(nx, ny, nz, storage, o);
    c->geo = make_geometry(nx, ny, nz, c->plan, storage);
    // When an iteration's vectors (r, p twice, x) exceed the last-level
    // cache, the update that adds to x (stencil, three axpys and a norm per
    // point) streams better with twice the planes per work-group while the
    // launch keeps at least 256 work-groups (256^3 FP32: 88.2 -> 83.6 us),
    // while the direction kernel and the update that leaves x stay faster
    // with the shorter chunk (36.4 against 45.6 us; 35.7 against 44.0 us).
    // With cache-resident vectors the taller chunk measured slower (192^3
    // FP32: 60.9 -> 62.7 us per iteration).
    c->plan_upd = c->plan;
    if (o.zchunk_update > 0) {
        c->plan_upd.zc = o.zchunk_update;
    } else if (o.zchunk_update == 0 && o.zchunk <= 0 &&
               (size_t)n * (3 * dt_size(storage) + dt_size(o.x_accum)) > LLC_BYTES) {
        Plan t = c->plan;
        t.zc = 2 * c->plan.zc;
        if (t.zc <= nz && make_geometry(nx, ny, nz, t, storage).nblocks >= 256) c->plan_upd = t;
    }
    c->geo_upd = make_geometry(nx, ny, nz, c->plan_upd, storage);
    c->plan_res = Plan{TILE_CFGS[c->plan.cfg].vec && (nx % 2 == 0) ? 2 : 5, c->plan.zc};
    c->geo_res = make_geometry(nx, ny, nz, c->plan_res, DT_F64);
    c->chunk_iters = o.chunk_iters;

    const size_t es = dt_size(storage);
    const size_t xs = dt_size(o.x_accum);
    size_t maxblk = std::max<size_t>({(size_t)c->geo.nblocks, (size_t)c->geo_upd.nblocks, (size_t)c->geo_res.nblocks,
                                      (size_t)DOT_MAX_BLOCKS});
    c->partials_cap = (size_t)MAX_RED_COMPONENTS * maxblk;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&c->r, es * n);
    if (e == hipSuccess) e = hipMalloc(&c->p[0], es * n);
    if (e == hipSuccess) e = hipMalloc(&c->p[1], es * n);
    if (e == hipSuccess) e = hipMalloc(&c->xacc, xs * n);
    if (e == hipSuccess) e = hipMalloc(&c->partials, sizeof(double) * c->partials_cap);
    if (e == hipSuccess) e = hipMalloc(&c->ticket, 256);
    if (e == hipSuccess) e = hipMalloc(&c->st, 2 * sizeof(SolveState));  // current state and the chain's second
    if (e == hipSuccess) e = hipMalloc(&c->res2, 2 * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(&c->hst, 2 * sizeof(SolveState), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&c->hres, 2 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_chunk[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_chunk[1], hipEventDisableTiming);
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(e == hipErrorOutOfMemory ? PCG_E_NOMEM : PCG_E_HIP, "pcg_create: %s", hipGetErrorString(e));
    }
    e = launch_zero(DT_F64, 32, c->ticket, c->stream);  // 256 bytes
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        free_ctx(c);
        return fail(PCG_E_HIP, "pcg_create: %s", hipGetErrorString(e));
    }
    pcg_status s = ensure_hist(c, 1023);
    if (s != PCG_OK) {
        free_ctx(c);
        return s;
    }
    *out = c;
    return PCG_OK;
}

pcg_status pcg_destroy(pcg_ctx c) {
    if (!c) return PCG_OK;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    return PCG_OK;
}

pcg_status stencil_apply(pcg_ctx c, const void* x, void* y) {
    if (!c) return fail(PCG_E_ARG, "stencil_apply: null context");
    if (!x || !y) return fail(PCG_E_ARG, "stencil_apply: null pointer");
    if (!aligned16(x) || !aligned16(y)) return fail(PCG_E_ARG, "stencil_apply: pointers must be 16-byte aligned");
    if (overlap(x, y, (size_t)c->n * dt_size(c->dt))) return fail(PCG_E_ARG, "stencil_apply: x and y overlap");
    HIPCHK(launch_stencil(c->dt, c->plan, c->geo, op_of(c), x, y, c->stream));
    return PCG_OK;
}

pcg_status axpy(pcg_ctx c, int64_t n, double alpha, const void* x, const void* y, void* z) {
    if (!c) return fail(PCG_E_ARG, "axpy: null context");
    if (n < 0) return fail(PCG_E_ARG, "axpy: negative length");
    if (n == 0) return PCG_OK;
    if (!x || !y || !z) return fail(PCG_E_ARG, "axpy: null pointer");
    if (!aligned16(x) || !aligned16(y) || !aligned16(z)) return fail(PCG_E_ARG, "axpy: pointers must be 16-byte aligned");
    const size_t bytes = (size_t)n * dt_size(c->dt);
    if ((z != x && overlap(z, x, bytes)) || (z != y && overlap(z, y, bytes)))
        return fail(PCG_E_ARG, "axpy: z partially overlaps an input");
    HIPCHK(launch_axpy(c->dt, n, alpha, x, y, z, c->stream));
    return PCG_OK;
}

static pcg_status dot_common(pcg_ctx c, int64_t n, const void* x, const void* y, float* of, double* od,
                             const char* name) {
    if (!c) return fail(PCG_E_ARG, "%s: null context", name);
    if (n < 0) return fail(PCG_E_ARG, "%s: negative length", name);
    if (!of && !od) return fail(PCG_E_ARG, "%s: null output", name);
    if (n > 0 && (!x || !y)) return fail(PCG_E_ARG, "%s: null pointer", name);
    if ((n > 0 && (!aligned16(x) || !aligned16(y))))
        return fail(PCG_E_ARG, "%s: pointers must be 16-byte aligned", name);
    HIPCHK(launch_dot(c->dt, n, x, y, of, od, red_of(c), c->stream));
    return PCG_OK;
}

pcg_status dot(pcg_ctx c, int64_t n, const void* x, const void* y, float* out_dev) {
    return dot_common(c, n, x, y, out_dev, nullptr, "dot");
}

pcg_status dot_f64(pcg_ctx c, int64_t n, const void* x, const void* y, double* out_dev) {
    return dot_common(c, n, x, y, nullptr, out_dev, "dot_f64");
}

pcg_status pcg_solve(pcg_ctx c, const void* b, void* x, double rtol, int maxit, pcg_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    Range range("pcg_solve");
    if (!c) return fail(PCG_E_ARG, "pcg_solve: null context");
    if (!b || !x) return fail(PCG_E_ARG, "pcg_solve: null pointer");
    if (!aligned16(b) || !aligned16(x)) return fail(PCG_E_ARG, "pcg_solve: pointers must be 16-byte aligned");
    if (!(rtol >= 0.0) || maxit < 0) return fail(PCG_E_ARG, "pcg_solve: rtol must be >= 0 and maxit >= 0");
    const size_t xbytes = (size_t)c->n * dt_size(c->opt.x_dtype);
    if (overlap2(b, (size_t)c->n * dt_size(c->dt), x, xbytes))
        return fail(PCG_E_ARG, "pcg_solve: b and x overlap");
    hipStream_t st = c->stream;
    const int xacc_dt = c->opt.x_accum;
    IterResult res;
    int restarts = 0, total_iters = 0;
    const void* x0 = c->opt.use_x0 ? x : nullptr;
    int x0_dt = c->opt.x_dtype;
    for (;;) {
        IterResult seg;  // run_iterations accumulates its kernel times into a fresh result
        pcg_status s;
        {
            Range r(restarts ? "PCG iterations (restart)" : "PCG iterations");
            s = run_iterations(c, b, x0, x0_dt, rtol, maxit - total_iters, 0, &seg);
        }
        if (s != PCG_OK) return s;
        total_iters += seg.fin.iters;
        res.k1_ms += seg.k1_ms;
        res.k2_ms += seg.k2_ms;
        res.nk += seg.nk;
        res.k2e_ms += seg.k2e_ms;
        res.nke += seg.nke;
        res.fin = seg.fin;

        // Result to the caller's x, then the FP64 true residual of what is returned.
        Range rr("FP64 true residual");
        if (c->opt.x_dtype == xacc_dt) HIPCHK(hipMemcpyAsync(x, c->xacc, xbytes, hipMemcpyDeviceToDevice, st));
        else HIPCHK(launch_convert(xacc_dt, c->opt.x_dtype, c->n, c->xacc, x, st));
        if (res.fin.rr0 == 0.0) HIPCHK(launch_zero(c->opt.x_dtype, c->n, x, st));
        HIPCHK(launch_residual64(c->dt, c->opt.x_dtype, c->plan_res, c->geo_res, op_of(c), b, x, c->res2, red_of(c),
                                 st));
        HIPCHK(hipMemcpyAsync(c->hres, c->res2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // Converged on the recursion but not in FP64: restart from the
        // accumulator with the FP64 residual (the start kernel recomputes it).
        const bool true_ok = c->hres[0] <= rtol * rtol * res.fin.rr0;
        if (res.fin.done != 1 || true_ok || restarts >= c->opt.max_restarts || total_iters >= maxit) break;
        ++restarts;
        x0 = c->xacc;
        x0_dt = xacc_dt;
    }
    res.fin.iters = total_iters;
    const SolveState& fin = res.fin;

    // The FP64 true residual of the returned x decides success.
    pcg_status ret = PCG_OK;
    if (fin.done == 2) ret = PCG_E_BREAKDOWN;
    else if (fin.done != 1) ret = PCG_E_NOCONV;
    else if (!(c->hres[0] <= rtol * rtol * fin.rr0)) ret = PCG_E_TRUE_RESIDUAL;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iters = fin.iters;
        info->status = ret;
        info->rel_res_recursive = fin.rr0 > 0 ? std::sqrt(fin.rr / fin.rr0) : 0.0;
        info->rel_res_true_fp64 = fin.rr0 > 0 ? std::sqrt(c->hres[0] / fin.rr0) : 0.0;
        info->k1_ms = res.k1_ms;
        info->k2_ms = res.k2_ms;
        info->k1_launches = res.nk;
        info->k2_launches = res.nk;
        info->k2_even_ms = res.k2e_ms;
        info->k2_even_launches = res.nke;
        info->restarts = restarts;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (ret == PCG_E_BREAKDOWN) fail(ret, "pcg_solve: breakdown (p.Ap <= 0 or a non-finite value) at iteration %d", fin.iters + 1);
    else if (ret == PCG_E_NOCONV) fail(ret, "pcg_solve: no convergence in %d iterations", maxit);
    else if (ret == PCG_E_TRUE_RESIDUAL)
        fail(ret, "pcg_solve: the recursion converged but the FP64 true residual %.3e is above rtol %.3e after %d restarts",
             info ? info->rel_res_true_fp64 : std::sqrt(c->hres[0] / fin.rr0), rtol, restarts);
    return ret;
}

pcg_status pcg_solve_refined(pcg_ctx c, const double* b64, double* x64, double rtol_outer, double rtol_inner,
                             int max_outer, int maxit_inner, pcg_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    Range range("pcg_solve_refined");
    if (!c) return fail(PCG_E_ARG, "pcg_solve_refined: null context");
    if (!b64 || !x64) return fail(PCG_E_ARG, "pcg_solve_refined: null pointer");
    if (!aligned16(b64) || !aligned16(x64)) return fail(PCG_E_ARG, "pcg_solve_refined: pointers must be 16-byte aligned");
    if (!(rtol_outer >= 0.0) || !(rtol_inner > 0.0) || max_outer < 0 || maxit_inner < 1)
        return fail(PCG_E_ARG, "pcg_solve_refined: bad tolerance or iteration limit");
    if (c->dt == DT_F64) return fail(PCG_E_UNSUPPORTED, "pcg_solve_refined: the inner storage must be F32, BF16 or F16");
    if (overlap(b64, x64, (size_t)c->n * 8)) return fail(PCG_E_ARG, "pcg_solve_refined: b and x overlap");
    hipStream_t st = c->stream;
    if (!c->rhat) HIPCHK(hipMalloc(&c->rhat, dt_size(c->dt) * c->n));
    const int xacc_dt = c->opt.x_accum;
    c->ref_relres.clear();
    c->ref_inner.clear();

    HIPCHK(launch_zero(DT_F64, c->n, x64, st));
    double nb = 0.0, t1e6 = -1.0, t1e10 = -1.0;
    int outer = 0, inner_total = 0;
    double k1_ms = 0.0, k2_ms = 0.0, k2e_ms = 0.0;  // kernel_timing: event-timed inner iteration kernels
    int nke = 0;
    int nk = 0;
    pcg_status ret = PCG_E_NOCONV;
    for (;;) {
        {
            Range r("refinement: FP64 residual");
            HIPCHK(launch_residual64(DT_F64, DT_F64, c->plan_res, c->geo_res, op_of(c), b64, x64, c->res2,
                                     red_of(c), st));
            HIPCHK(hipMemcpyAsync(c->hres, c->res2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        const double rn = std::sqrt(c->hres[0]), amax = c->hres[1];
        if (outer == 0) nb = rn;  // x = 0: the residual is b
        const double t = nb > 0.0 ? rn / nb : 0.0;
        const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        c->ref_relres.push_back(t);
        if (!std::isfinite(t)) {
            ret = PCG_E_BREAKDOWN;
            break;
        }
        if (t <= 1e-6 && t1e6 < 0) t1e6 = now;
        if (t <= 1e-10 && t1e10 < 0) t1e10 = now;
        if (t <= rtol_outer) {
            ret = PCG_OK;
            break;
        }
        if (outer >= max_outer) break;
        // rhat = lp(s (b - A x)), s = 1 / max|r|; inner Jacobi-PCG A d = rhat.
        const double scale = 1.0 / amax;
        HIPCHK(launch_cast_scaled(c->dt, c->plan_res, c->geo_res, op_of(c), b64, x64, scale, c->rhat, st));
        IterResult res;
        pcg_status s;
        {
            Range r("refinement: low-precision inner solve");
            s = run_iterations(c, c->rhat, nullptr, c->dt, rtol_inner, maxit_inner, c->opt.stag_window, &res);
        }
        if (s != PCG_OK) return s;
        c->ref_inner.push_back(res.fin.iters);
        inner_total += res.fin.iters;
        k1_ms += res.k1_ms;
        k2_ms += res.k2_ms;
        nk += res.nk;
        k2e_ms += res.k2e_ms;
        nke += res.nke;
        HIPCHK(launch_correct(xacc_dt, c->n, c->xacc, scale, x64, st));
        ++outer;
    }
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iters = inner_total;
        info->outer_iters = outer;
        info->status = ret;
        info->rel_res_true_fp64 = c->ref_relres.empty() ? 0.0 : c->ref_relres.back();
        info->rel_res_recursive = info->rel_res_true_fp64;
        info->t_1e6 = t1e6;
        info->t_1e10 = t1e10;
        info->k1_ms = k1_ms;
        info->k2_ms = k2_ms;
        info->k2_even_ms = k2e_ms;
        info->k2_even_launches = nke;
        info->k1_launches = nk;
        info->k2_launches = nk;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (ret == PCG_E_NOCONV) fail(ret, "pcg_solve_refined: not converged after %d refinement steps", outer);
    else if (ret == PCG_E_BREAKDOWN) fail(ret, "pcg_solve_refined: non-finite residual");
    return ret;
}

pcg_status pcg_refine_history(pcg_ctx c, double* relres, int* inner_iters, int n, int* count) {
    if (!c || !count || n < 0) return fail(PCG_E_ARG, "pcg_refine_history: bad argument");
    int m = std::min<int>(n, (int)c->ref_relres.size());
    for (int i = 0; i < m; ++i) {
        if (relres) relres[i] = c->ref_relres[i];
        if (inner_iters) inner_iters[i] = i < (int)c->ref_inner.size() ? c->ref_inner[i] : 0;
    }
    *count = m;
    return PCG_OK;
}

// Flexible CG with the network's preconditioner (net), the multigrid
// V-cycle (mg) or Jacobi (neither); `name` prefixes error messages.
static pcg_status flex_solve(pcg_ctx c, cnn_net net, bool mg, const float* g, const void* b, void* x, double rtol,
                             int maxit, pcg_info* info, const char* name) {
    auto t0 = std::chrono::steady_clock::now();
    Range range(name);
    if (!c) return fail(PCG_E_ARG, "%s: null context", name);
    if (!b || !x) return fail(PCG_E_ARG, "%s: null pointer", name);
    if (!aligned16(b) || !aligned16(x)) return fail(PCG_E_ARG, "%s: pointers must be 16-byte aligned", name);
    if (!(rtol >= 0.0) || maxit < 0) return fail(PCG_E_ARG, "%s: rtol must be >= 0 and maxit >= 0", name);
    if (c->dt != DT_F32 || c->opt.x_accum != DT_F64)
        return fail(PCG_E_UNSUPPORTED, "%s: needs F32 storage with an FP64 x accumulator", name);
    if (net && cnn_stream_of(net) != c->stream)
        return fail(PCG_E_ARG, "%s: the network and the context must use the same stream", name);
    const size_t xbytes = (size_t)c->n * dt_size(c->opt.x_dtype);
    if (overlap2(b, (size_t)c->n * 4, x, xbytes)) return fail(PCG_E_ARG, "%s: b and x overlap", name);
    pcg_status s = ensure_hist(c, maxit);
    if (s != PCG_OK) return s;
    hipStream_t st = c->stream;
    if (!c->q) HIPCHK(hipMalloc(&c->q, 4 * c->n));
    if (!c->z) HIPCHK(hipMalloc(&c->z, 4 * c->n));
    const OpDesc od = op_of(c);
    const float* dinv = static_cast<const float*>(od.dinv);
    float* r = static_cast<float*>(c->r);
    float* q = static_cast<float*>(c->q);
    float* z = static_cast<float*>(c->z);
    double* xacc = static_cast<double*>(c->xacc);

    // With two or more levels the V-cycle's last sweep also does the select
    // step (saves a pass over z, r and q per iteration).
    const bool mg_fused = mg && c->mg && c->mg->nlev >= 2;
    auto precond = [&](bool use_net) -> pcg_status {
        if (use_net) {
            pcg_status ps = cnn_forward(net, c->nx, c->ny, c->nz, PCG_F32, r, g, &c->st->rr, z);
            if (ps != PCG_OK) return ps;
        }
        if (mg_fused) {  // the V-cycle's last sweep does the select step
            const MgSelect sel{q, c->st, red_of(c)};
            HIPCHK(launch_mg_vcycle(*c->mg, r, z, &c->st->done, st, &sel));
        } else {
            if (mg) HIPCHK(launch_mg_vcycle(*c->mg, r, z, &c->st->done, st));
            HIPCHK(launch_flex_select(c->n, z, r, q, dinv, c->st, false, red_of(c), st));
        }
        HIPCHK(launch_flex_select(c->n, z, r, q, dinv, c->st, true, red_of(c), st));
        return PCG_OK;
    };
    bool net_on = net != nullptr;
    bool mg_on = mg;
    // Start of a run of iterations: from x = 0, or (a restart) from the
    // accumulator with r = fl32(b - A x) computed in FP64.
    auto start_segment = [&](bool from_x, int seg_maxit) -> pcg_status {
        SolveState init{};
        init.tol2 = rtol * rtol;
        init.dinv = 1.0 / 6.0;
        init.maxit = seg_maxit;
        init.stag = FLEX_STAG_WINDOW;
        init.flags = FLEX_RESTART | (net || mg ? 0 : FLEX_JACOBI) | (mg ? FLEX_MG : 0);
        init.fallback_at = -1;
        c->hst[0] = init;
        HIPCHK(hipMemcpyAsync(c->st, &c->hst[0], sizeof(SolveState), hipMemcpyHostToDevice, st));
        if (from_x)
            HIPCHK(launch_pcg_start_x0(DT_F32, DT_F64, c->plan_res, c->geo_res, od, b, xacc, r, c->st, c->hist,
                                       red_of(c), st));
        else
            HIPCHK(launch_pcg_start_zero(DT_F32, c->n, b, r, xacc, DT_F64, c->p[0], od.dinv, c->st, c->hist,
                                         red_of(c), st));
        HIPCHK(launch_zero(DT_F32, c->n, q, st));
        return precond(net_on);
    };
    s = start_segment(false, maxit);
    if (s != PCG_OK) return s;

    // Iterations k = 1..C of a chunk (C even, so iteration parity repeats) on
    // stream s; the network launches on its own stream, swapped to s. The
    // multigrid iteration converges in ~10-15 iterations and launches ~30
    // kernels per iteration: chunks of 4 keep the launches past convergence
    // (each returns at once but costs its launch) few.
    const int C = mg ? std::min(c->chunk_iters, 4) : c->chunk_iters;
    auto enqueue_chunk = [&](bool use_net, bool use_mg, hipStream_t sq) -> pcg_status {
        for (int k = 1; k <= C; ++k) {
            void* pold = c->p[(k - 1) & 1];
            void* pnew = c->p[k & 1];
            HIPCHK(launch_flex_direction(c->plan, c->geo, od, z, static_cast<const float*>(pold),
                                         static_cast<float*>(pnew), q, r, c->st, red_of(c), sq));
            HIPCHK(launch_flex_update(c->n, static_cast<const float*>(pnew), static_cast<const float*>(pold), q, r,
                                      xacc, c->st, c->hist, red_of(c), sq));
            if (use_net) {
                pcg_status ps = cnn_forward(net, c->nx, c->ny, c->nz, PCG_F32, r, g, &c->st->rr, z);
                if (ps != PCG_OK) return ps;
            }
            if (use_mg && mg_fused) {
                const MgSelect sel{q, c->st, red_of(c)};
                HIPCHK(launch_mg_vcycle(*c->mg, r, z, &c->st->done, sq, &sel));
            } else {
                if (use_mg) HIPCHK(launch_mg_vcycle(*c->mg, r, z, &c->st->done, sq));
                HIPCHK(launch_flex_select(c->n, z, r, q, dinv, c->st, false, red_of(c), sq));
            }
            HIPCHK(launch_flex_select(c->n, z, r, q, dinv, c->st, true, red_of(c), sq));
        }
        return PCG_OK;
    };
    // A chunk is replayed from a captured graph (recorded once per network,
    // field, workspace and operator): the flexible iteration is ~9 launches,
    // latency-bound on small grids. Kernels after convergence or a switch to
    // Jacobi skip their work on the device state, as in the eager loop.
    uint64_t epoch = 0;
    if (net) {
        s = cnn_prepare(net, c->nx, c->ny, c->nz, &epoch);
        if (s != PCG_OK) return s;
    }
    auto chunk_graph = [&](bool use_net, bool use_mg, hipGraphExec_t* out) -> pcg_status {
        const int slot = use_mg ? 2 : use_net ? 1 : 0;
        const pcg_ctx_s::FlexKey key{use_net ? net : nullptr, use_net ? g : nullptr, use_net ? epoch : 0, c->hist,
                                     c->kc, C, use_mg ? c->mg_epoch : 0};
        auto& have = c->flex_key[slot];
        if (c->flex_exec[slot] && have.net == key.net && have.g == key.g && have.epoch == key.epoch &&
            have.hist == key.hist && have.kc == key.kc && have.chunk == key.chunk && have.mg_epoch == key.mg_epoch) {
            *out = c->flex_exec[slot];
            return PCG_OK;
        }
        if (c->flex_exec[slot]) {
            HIPCHK(hipGraphExecDestroy(c->flex_exec[slot]));
            c->flex_exec[slot] = nullptr;
        }
        Range range("graph capture: flexible iterations");
        if (!c->capture) HIPCHK(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
        hipStream_t old = use_net ? cnn_swap_stream(net, c->capture) : nullptr;
        hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
        pcg_status ps = e == hipSuccess ? enqueue_chunk(use_net, use_mg, c->capture) : PCG_E_HIP;
        hipGraph_t gr = nullptr;
        hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->capture, &gr) : e;
        if (use_net) (void)cnn_swap_stream(net, old);
        if (ps != PCG_OK || e2 != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return ps != PCG_OK ? ps : fail(PCG_E_HIP, "capturing flexible iterations failed: %s", hipGetErrorString(e2));
        }
        hipError_t e3 = hipGraphInstantiate(&c->flex_exec[slot], gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e3 != hipSuccess) {
            c->flex_exec[slot] = nullptr;
            return fail(PCG_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
        }
        have = key;
        *out = c->flex_exec[slot];
        return PCG_OK;
    };

    SolveState fin{};
    const bool graph = c->opt.use_graph && !c->opt.kernel_timing;
    auto iterate = [&](int seg_maxit) -> pcg_status {
        Range r("flexible iterations");
        int it = 0;
        for (;;) {
            HIPCHK(hipMemcpyAsync(&c->hst[1], c->st, sizeof(SolveState), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            fin = c->hst[1];
            if (fin.done != 0 || it >= seg_maxit) break;
            if (fin.flags & FLEX_JACOBI) net_on = mg_on = false;
            if (graph) {
                hipGraphExec_t ge = nullptr;
                pcg_status ps = chunk_graph(net_on, mg_on, &ge);
                if (ps != PCG_OK) return ps;
                HIPCHK(hipGraphLaunch(ge, st));
            } else {
                pcg_status ps = enqueue_chunk(net_on, mg_on, st);
                if (ps != PCG_OK) return ps;
            }
            it += C;
        }
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(&fin, c->st, sizeof(SolveState), hipMemcpyDeviceToHost));
        // x advances every second iteration: after an odd count it still
        // owes the last step (direction in p[1], alpha in the state)
        if (fin.iters & 1) {
            HIPCHK(launch_x_finish(DT_F32, DT_F64, c->n, xacc, c->p[1], c->st, false, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        return PCG_OK;
    };
    auto true_residual = [&](double* rel) -> pcg_status {
        Range r("FP64 true residual");
        HIPCHK(launch_residual64(DT_F32, DT_F64, c->plan_res, c->geo_res, od, b, xacc, c->res2, red_of(c), st));
        HIPCHK(hipMemcpyAsync(c->hres, c->res2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *rel = fin.rr0 > 0 ? std::sqrt(c->hres[0] / fin.rr0) : 0.0;
        return PCG_OK;
    };
    s = iterate(maxit);
    if (s != PCG_OK) return s;
    int iters = fin.iters;
    int fallback = fin.fallback_at >= 0 ? 1 : 0;
    int status = fin.done;

    // The FP64 true residual judges the result. With the V-cycle, a converged
    // recursion whose true residual is above rtol restarts the same method
    // from x with r = fl32(b - A x) (at most max_restarts times); otherwise
    // Jacobi-PCG continues from this x.
    double true_rel = 0.0;
    s = true_residual(&true_rel);
    if (s != PCG_OK) return s;
    int restarts = 0;
    while (mg && status == 1 && true_rel > rtol && iters < maxit && restarts < c->opt.max_restarts) {
        ++restarts;
        mg_on = true;
        s = start_segment(true, maxit - iters);
        if (s != PCG_OK) return s;
        s = iterate(maxit - iters);
        if (s != PCG_OK) return s;
        iters += fin.iters;
        status = fin.done;
        if (fin.fallback_at >= 0) fallback = 1;
        s = true_residual(&true_rel);
        if (s != PCG_OK) return s;
    }
    if (!mg && status == 1 && true_rel > rtol && iters < maxit) {
        Range r("Jacobi-PCG continuation");
        IterResult res;
        s = run_iterations(c, b, xacc, DT_F64, rtol, maxit - iters, 0, &res);
        if (s != PCG_OK) return s;
        iters += res.fin.iters;
        status = res.fin.done;
        fallback = 2;
        HIPCHK(launch_residual64(DT_F32, DT_F64, c->plan_res, c->geo_res, od, b, xacc, c->res2, red_of(c), st));
        HIPCHK(hipMemcpyAsync(c->hres, c->res2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        true_rel = fin.rr0 > 0 ? std::sqrt(c->hres[0] / fin.rr0) : 0.0;
        fin.rr = res.fin.rr;
    }
    if (c->opt.x_dtype == DT_F64) HIPCHK(hipMemcpyAsync(x, xacc, xbytes, hipMemcpyDeviceToDevice, st));
    else HIPCHK(launch_convert(DT_F64, c->opt.x_dtype, c->n, xacc, x, st));
    HIPCHK(hipStreamSynchronize(st));
    c->last_iters = fin.iters;
    pcg_status ret = status == 1 ? (true_rel <= rtol ? PCG_OK : PCG_E_TRUE_RESIDUAL)
                   : status == 2 ? PCG_E_BREAKDOWN : PCG_E_NOCONV;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iters = iters;
        info->status = ret;
        info->fallback_used = fallback;
        info->outer_iters = fin.fallback_at;
        info->rel_res_recursive = fin.rr0 > 0 ? std::sqrt(fin.rr / fin.rr0) : 0.0;
        info->rel_res_true_fp64 = true_rel;
        info->restarts = restarts;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (ret == PCG_E_BREAKDOWN) fail(ret, "%s: breakdown", name);
    else if (ret == PCG_E_NOCONV) fail(ret, "%s: no convergence in %d iterations", name, maxit);
    else if (ret == PCG_E_TRUE_RESIDUAL)
        fail(ret, "%s: the FP64 true residual %.3e is above rtol %.3e", name, true_rel, rtol);
    return ret;
}

pcg_status pcg_solve_flexible(pcg_ctx c, cnn_net net, const float* g, const void* b, void* x, double rtol,
                              int maxit, pcg_info* info) {
    return flex_solve(c, net, false, g, b, x, rtol, maxit, info, "pcg_solve_flexible");
}

pcg_status pcg_solve_mg(pcg_ctx c, const void* b, void* x, double rtol, int maxit, pcg_info* info) {
    if (!c) return fail(PCG_E_ARG, "pcg_solve_mg: null context");
    if (!c->mg) return fail(PCG_E_ARG, "pcg_solve_mg: no multigrid hierarchy (call pcg_set_multigrid first)");
    return flex_solve(c, nullptr, true, nullptr, b, x, rtol, maxit, info, "pcg_solve_mg");
}

pcg_status pcg_solve_snapshots(pcg_ctx c, const void* b, void* x, double rtol, int maxit, const int* snap_iters,
                               int nsnap, void* r_snaps, void* x_snaps, pcg_info* info) {
    if (!c || !b || !x || (nsnap > 0 && (!snap_iters || !r_snaps || !x_snaps)))
        return fail(PCG_E_ARG, "pcg_solve_snapshots: null argument");
    if (nsnap < 0 || maxit < 0 || !(rtol >= 0.0)) return fail(PCG_E_ARG, "pcg_solve_snapshots: bad count");
    for (int j = 1; j < nsnap; ++j)
        if (snap_iters[j] <= snap_iters[j - 1]) return fail(PCG_E_ARG, "pcg_solve_snapshots: iterations must increase");
    if (c->opt.x_dtype != c->opt.x_accum)
        return fail(PCG_E_ARG, "pcg_solve_snapshots: x_dtype must equal the accumulator type");
    pcg_status s = ensure_hist(c, maxit);
    if (s != PCG_OK) return s;
    hipStream_t st = c->stream;
    const size_t es = dt_size(c->dt), xs = dt_size(c->opt.x_accum);
    SolveState init{};
    init.tol2 = rtol * rtol;
    init.dinv = 1.0 / 6.0;
    init.maxit = maxit;
    c->hst[0] = init;
    HIPCHK(hipMemcpyAsync(c->st, &c->hst[0], sizeof(SolveState), hipMemcpyHostToDevice, st));
    c->sr_active = false;  // snapshots step one two-kernel iteration at a time
    HIPCHK(launch_pcg_start_zero(c->dt, c->n, b, c->r, c->xacc, c->opt.x_accum, c->p[0], op_of(c).dinv, c->st,
                                 c->hist, red_of(c), st));
    int j = 0;
    SolveState fin{};
    for (int it = 1; it <= maxit; ++it) {
        hipError_t e = enqueue_iters(c, it, 1, st, nullptr, true);
        if (e != hipSuccess) return fail(PCG_E_HIP, "pcg_solve_snapshots: %s", hipGetErrorString(e));
        while (j < nsnap && snap_iters[j] == it) {
            HIPCHK(hipMemcpyAsync(static_cast<char*>(r_snaps) + (size_t)j * c->n * es, c->r, c->n * es,
                                  hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(static_cast<char*>(x_snaps) + (size_t)j * c->n * xs, c->xacc, c->n * xs,
                                  hipMemcpyDeviceToDevice, st));
            ++j;
        }
        if (it % 32 == 0 || it == maxit) {
            HIPCHK(hipMemcpyAsync(&c->hst[1], c->st, sizeof(SolveState), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (c->hst[1].done != 0 && j >= nsnap) break;
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(&fin, c->st, sizeof(SolveState), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpyAsync(x, c->xacc, c->n * xs, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    c->last_iters = fin.iters;
    const pcg_status ret = fin.done == 1 ? PCG_OK : fin.done == 2 ? PCG_E_BREAKDOWN : PCG_E_NOCONV;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->iters = fin.iters;
        info->status = ret;
        info->rel_res_recursive = fin.rr0 > 0 ? std::sqrt(fin.rr / fin.rr0) : 0.0;
    }
    if (ret != PCG_OK) fail(ret, "pcg_solve_snapshots: solve did not converge (status %d)", (int)ret);
    return ret;
}

pcg_status pcg_make_pairs(pcg_ctx c, int npairs, const double* r_snaps, const double* x_snaps, const double* x_star,
                          void* pairs) {
    if (!c || npairs < 0 || (npairs > 0 && (!r_snaps || !x_snaps || !x_star || !pairs)))
        return fail(PCG_E_ARG, "pcg_make_pairs: bad argument");
    hipStream_t st = c->stream;
    for (int j = 0; j < npairs; ++j) {
        const double* rj = r_snaps + (size_t)j * c->n;
        HIPCHK(launch_dot(DT_F64, c->n, rj, rj, nullptr, c->res2, red_of(c), st));
        HIPCHK(launch_make_pair(c->n, rj, x_snaps + (size_t)j * c->n, x_star, c->res2,
                                static_cast<uint16_t*>(pairs) + (size_t)2 * j * c->n, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return PCG_OK;
}

pcg_status pcg_set_coefficients(pcg_ctx c, const float* k_cell) {
    if (!c) return fail(PCG_E_ARG, "pcg_set_coefficients: null context");
    if (!k_cell) {
        c->kc = nullptr;
        if (c->chunk) {
            HIPCHK(hipGraphExecDestroy(c->chunk));
            c->chunk = nullptr;
        }
        if (c->mg) return build_mg(c);
        return PCG_OK;
    }
    if (!aligned16(k_cell)) return fail(PCG_E_ARG, "pcg_set_coefficients: k must be 16-byte aligned");
    if (c->dt != DT_F32 && c->dt != DT_F64)
        return fail(PCG_E_UNSUPPORTED, "pcg_set_coefficients: variable coefficients need F32 or F64 storage");
    if (!c->dinv) HIPCHK(hipMalloc(&c->dinv, dt_size(c->dt) * c->n));
    HIPCHK(launch_var_dinv(c->dt, c->plan, c->geo, k_cell, c->dinv, c->stream));
    c->kc = k_cell;
    if (c->chunk) {  // captured kernels use the old operator
        HIPCHK(hipGraphExecDestroy(c->chunk));
        c->chunk = nullptr;
    }
    if (c->mg) return build_mg(c);  // the hierarchy follows the operator
    return PCG_OK;
}

pcg_status pcg_set_multigrid(pcg_ctx c, int nu, double omega, int coarse_max) {
    if (!c) return fail(PCG_E_ARG, "pcg_set_multigrid: null context");
    if (nu < 1 || nu > 8) return fail(PCG_E_ARG, "pcg_set_multigrid: nu must be in 1..8 (got %d)", nu);
    if (omega == 0.0) omega = 6.0 / 7.0;
    if (!(omega > 0.0 && omega <= 1.0)) return fail(PCG_E_ARG, "pcg_set_multigrid: omega must be in (0, 1]");
    if (coarse_max < 0) return fail(PCG_E_ARG, "pcg_set_multigrid: coarse_max must be >= 0");
    if (c->dt != DT_F32) return fail(PCG_E_UNSUPPORTED, "pcg_set_multigrid: needs F32 storage");
    c->mg_nu = nu;
    c->mg_omega = omega;
    c->mg_coarse_max = coarse_max == 0 ? 512 : coarse_max;
    return build_mg(c);
}

pcg_status pcg_mg_apply(pcg_ctx c, const float* g, float* u) {
    if (!c) return fail(PCG_E_ARG, "pcg_mg_apply: null context");
    if (!c->mg) return fail(PCG_E_ARG, "pcg_mg_apply: no multigrid hierarchy (call pcg_set_multigrid first)");
    if (!g || !u) return fail(PCG_E_ARG, "pcg_mg_apply: null pointer");
    if (!aligned16(g) || !aligned16(u)) return fail(PCG_E_ARG, "pcg_mg_apply: pointers must be 16-byte aligned");
    if (overlap(g, u, sizeof(float) * (size_t)c->n)) return fail(PCG_E_ARG, "pcg_mg_apply: g and u overlap");
    HIPCHK(launch_mg_vcycle(*c->mg, g, u, c->zero_flag, c->stream));
    return PCG_OK;
}

pcg_status pcg_mg_levels(pcg_ctx c, int* nlev, int* dims) {
    if (!c || !nlev) return fail(PCG_E_ARG, "pcg_mg_levels: null argument");
    if (!c->mg) return fail(PCG_E_ARG, "pcg_mg_levels: no multigrid hierarchy (call pcg_set_multigrid first)");
    *nlev = c->mg->nlev;
    if (dims)
        for (int l = 0; l < c->mg->nlev; ++l) {
            dims[3 * l] = c->mg->lv[l].nx;
            dims[3 * l + 1] = c->mg->lv[l].ny;
            dims[3 * l + 2] = c->mg->lv[l].nz;
        }
    return PCG_OK;
}

pcg_status pcg_get_history(pcg_ctx c, double* hist, int n, int* count) {
    if (!c || !hist || !count || n < 0) return fail(PCG_E_ARG, "pcg_get_history: bad argument");
    int m = std::min(n, c->last_iters + 1);
    m = std::min(m, c->hist_cap);
    HIPCHK(hipMemcpy(hist, c->hist, sizeof(double) * m, hipMemcpyDeviceToHost));
    *count = m;
    return PCG_OK;
}

}  // extern "C"
