// cnn_api.hip -- the learned preconditioner's network object and its C ABI:
// weights (FP32 master, BF16 swizzled copies for the matrix cores),
// activations sized for the grid in use, inference z = rms(r) N(r / rms(r), g)
// and the training step (loss, back-propagation, Adam).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "pcgmi.h"
#include "trace.hpp"

using namespace pcgmi;

namespace pcgmi {
hipError_t launch_conv3d(int nx, int ny, int nz, int cin, int mode, const void* in, const void* wsw, void* out,
                         const void* mask, const double* scale_rms2, double scale_mul, const void* zeros, void* sink,
                         hipStream_t s);
hipError_t launch_conv3d_input(int nx, int ny, int nz, int dt, const void* r, const float* g, const double* rr,
                               const void* wsw, void* out, const void* zeros, void* sink, hipStream_t s);
hipError_t launch_pack_input(int dt, int64_t n, const void* r, const float* g, const double* rr, void* out,
                             hipStream_t s);
hipError_t launch_swizzle_weights(const float* w, int cin, int cout, int CIN, int mirror, void* out, hipStream_t s);
int conv_swizzle_elems(int CIN);
int conv_sink_bytes();
int wgrad_groups(int nx, int ny, int nz);
hipError_t launch_wgrad(int nx, int ny, int nz, int cx, int cy, const void* X, const void* dY, bool dy_f32,
                        const void* zeros, float* partials, int groups, hipStream_t s);
hipError_t launch_reduce_partials(const float* partials, int groups, int len, float scale, bool accumulate,
                                  float* grad, hipStream_t s);
hipError_t launch_loss(int64_t n, const float* out, const void* tgt, double* loss_acc, double* coef, float* dout,
                       void* dpack, Red red, hipStream_t s);
hipError_t launch_adam(int n, float* w, const float* g, float* m, float* v, float lr, int step, hipStream_t s);
hipError_t launch_anorm_u(int64_t n, const float* out, const void* pair, const float* dinv, float* u, hipStream_t s);
hipError_t launch_anorm_loss(int64_t n, const float* u, const float* au, const void* rh, bool energy,
                             const float* dinv, double* loss_acc, double* coef, float* dout, void* dpack, Red red,
                             hipStream_t s);
hipError_t ctx_apply_f32(pcg_ctx c, const float* u, float* y);
const float* ctx_dinv_f32(pcg_ctx c);
bool ctx_is_f32_grid(pcg_ctx c, int nx, int ny, int nz);
hipStream_t ctx_stream(pcg_ctx c);
const char* set_error(pcg_status st, const char* msg);
}  // namespace pcgmi

namespace {

// Layer shapes: 2 -> 16 -> 16 -> 16 -> 1; offsets into the packed weight vector.
constexpr int NL = 4;
constexpr int CIN[NL] = {2, 16, 16, 16};
constexpr int COUT[NL] = {16, 16, 16, 1};
constexpr int WOFF[NL + 1] = {0, 864, 7776, 14688, 15120};
constexpr int NW = 15120;
enum { OUT_RELU = 0, OUT_SCALED = 1, OUT_MASK = 2 };

pcg_status err(pcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(st, buf);
    return st;
}

#define CHK(expr)                                                                                         \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return err(PCG_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct cnn_s {
    hipStream_t stream = nullptr;
    float *w = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    void* wf[NL] = {};  // forward swizzles
    void* wb[NL] = {};  // input-gradient swizzles (layers 1..3 use the next layer's mirrored weights)
    bool dirty = true;
    int step = 0;
    // grid workspace
    int nx = 0, ny = 0, nz = 0;
    int64_t nvox = 0;
    void *in0 = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *da = nullptr, *db = nullptr;
    float *out = nullptr, *dout = nullptr, *partials = nullptr;
    void* dpack = nullptr;
    int groups = 0;
    double* scal = nullptr;  // {loss accumulator, gradient coefficient}
    double* rpart = nullptr;
    void* zeros = nullptr;  // 64 zero bytes: read in place of points outside the grid
    void* sink = nullptr;   // written in place of outputs outside the grid (never read)
    unsigned* ticket = nullptr;
    // A-norm loss: the operator's context (null: relative-MSE loss) and
    // the vectors u = N + D^-1 rh - eh and A u
    pcg_ctx op = nullptr;
    bool energy = false;  // normaliser rh.eh (the error's energy) instead of rh.D^-1 rh
    float *u = nullptr, *au = nullptr;
    uint64_t grid_epoch = 0;  // bumped whenever the grid workspace is reallocated
};

namespace {

void free_grid(cnn_net n) {
    void* p[] = {n->in0, n->h1, n->h2, n->h3, n->da, n->db, n->out, n->dout, n->partials, n->dpack, n->u, n->au};
    for (void* q : p)
        if (q) (void)hipFree(q);
    n->in0 = n->h1 = n->h2 = n->h3 = n->da = n->db = n->dpack = nullptr;
    n->out = n->dout = n->partials = n->u = n->au = nullptr;
    n->nvox = 0;
}

pcg_status ensure_grid(cnn_net n, int nx, int ny, int nz) {
    if (nx == n->nx && ny == n->ny && nz == n->nz && n->nvox) return PCG_OK;
    CHK(hipStreamSynchronize(n->stream));
    free_grid(n);
    const int64_t nv = (int64_t)nx * ny * nz;
    n->groups = wgrad_groups(nx, ny, nz);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&n->in0, 4 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->h1, 32 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->h2, 32 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->h3, 32 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->da, 32 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->db, 32 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->out, 4 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->dout, 4 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->dpack, 4 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->partials, sizeof(float) * (size_t)n->groups * 27 * 256);
    if (e == hipSuccess) e = hipMalloc(&n->u, 4 * nv);
    if (e == hipSuccess) e = hipMalloc(&n->au, 4 * nv);
    if (e != hipSuccess) {
        free_grid(n);
        return err(e == hipErrorOutOfMemory ? PCG_E_NOMEM : PCG_E_HIP, "cnn: workspace: %s", hipGetErrorString(e));
    }
    n->nx = nx;
    n->ny = ny;
    n->nz = nz;
    n->nvox = nv;
    ++n->grid_epoch;
    return PCG_OK;
}

pcg_status ensure_swizzled(cnn_net n) {
    if (!n->dirty) return PCG_OK;
    for (int l = 0; l < NL; ++l)
        CHK(launch_swizzle_weights(n->w + WOFF[l], CIN[l], COUT[l], CIN[l] == 2 ? 2 : 16, 0, n->wf[l], n->stream));
    // input gradient of layer l's input goes through layer l's mirrored weights:
    // wb[l] for l = 1..3 (layer 4's input gradient has 1 input channel -> packed width 2)
    for (int l = 1; l < NL; ++l)
        CHK(launch_swizzle_weights(n->w + WOFF[l], CIN[l], COUT[l], COUT[l] == 1 ? 2 : 16, 1, n->wb[l], n->stream));
    n->dirty = false;
    return PCG_OK;
}

// Forward through the four layers from n->in0 (or, with first_done, from
// layer 1's output already in n->h1); the last layer writes `out` scaled by
// sqrt(*rr) * mul (or mul when rr is null).
pcg_status forward(cnn_net n, float* out, const double* rr, double mul, bool first_done = false) {
    const int X = n->nx, Y = n->ny, Z = n->nz;
    hipStream_t s = n->stream;
    if (!first_done)
        CHK(launch_conv3d(X, Y, Z, 2, OUT_RELU, n->in0, n->wf[0], n->h1, nullptr, nullptr, 1.0, n->zeros, n->sink, s));
    CHK(launch_conv3d(X, Y, Z, 16, OUT_RELU, n->h1, n->wf[1], n->h2, nullptr, nullptr, 1.0, n->zeros, n->sink, s));
    CHK(launch_conv3d(X, Y, Z, 16, OUT_RELU, n->h2, n->wf[2], n->h3, nullptr, nullptr, 1.0, n->zeros, n->sink, s));
    CHK(launch_conv3d(X, Y, Z, 16, OUT_SCALED, n->h3, n->wf[3], out, nullptr, rr, mul, n->zeros, n->sink, s));
    return PCG_OK;
}

}  // namespace

namespace pcgmi {
hipStream_t cnn_stream_of(cnn_net n) { return n->stream; }
// The stream the network launches on (a capturing stream while a solver
// records a graph of its iterations); returns the previous one.
hipStream_t cnn_swap_stream(cnn_net n, hipStream_t s) {
    hipStream_t old = n->stream;
    n->stream = s;
    return old;
}
// Grid workspace and swizzled weights ready for nx x ny x nz (nothing is
// allocated or launched later by cnn_forward on that grid until the weights
// change); *epoch identifies the workspace's buffers.
pcg_status cnn_prepare(cnn_net n, int nx, int ny, int nz, uint64_t* epoch) {
    pcg_status st = ensure_grid(n, nx, ny, nz);
    if (st != PCG_OK) return st;
    st = ensure_swizzled(n);
    if (st != PCG_OK) return st;
    *epoch = n->grid_epoch;
    return PCG_OK;
}
}  // namespace pcgmi

extern "C" {

pcg_status cnn_create(cnn_net* out, void* hip_stream) {
    if (!out) return err(PCG_E_ARG, "cnn_create: null output handle");
    *out = nullptr;
    cnn_net n = new (std::nothrow) cnn_s();
    if (!n) return err(PCG_E_NOMEM, "cnn_create: out of host memory");
    n->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&n->w, sizeof(float) * NW);
    if (e == hipSuccess) e = hipMalloc(&n->grad, sizeof(float) * NW);
    if (e == hipSuccess) e = hipMalloc(&n->m, sizeof(float) * NW);
    if (e == hipSuccess) e = hipMalloc(&n->v, sizeof(float) * NW);
    for (int l = 0; l < NL && e == hipSuccess; ++l)
        e = hipMalloc(&n->wf[l], 2 * conv_swizzle_elems(CIN[l] == 2 ? 2 : 16));
    for (int l = 1; l < NL && e == hipSuccess; ++l)
        e = hipMalloc(&n->wb[l], 2 * conv_swizzle_elems(COUT[l] == 1 ? 2 : 16));
    if (e == hipSuccess) e = hipMalloc(&n->scal, 4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&n->rpart, sizeof(double) * 2 * DOT_MAX_BLOCKS);
    if (e == hipSuccess) e = hipMalloc(&n->ticket, 256);
    if (e == hipSuccess) e = hipMalloc(&n->zeros, 64);
    if (e == hipSuccess) e = hipMemsetAsync(n->zeros, 0, 64, n->stream);
    if (e == hipSuccess) e = hipMalloc(&n->sink, conv_sink_bytes());
    if (e == hipSuccess) e = hipMemsetAsync(n->w, 0, sizeof(float) * NW, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->m, 0, sizeof(float) * NW, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->v, 0, sizeof(float) * NW, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->ticket, 0, 256, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) {
        cnn_destroy(n);
        return err(PCG_E_HIP, "cnn_create: %s", hipGetErrorString(e));
    }
    *out = n;
    return PCG_OK;
}

pcg_status cnn_destroy(cnn_net n) {
    if (!n) return PCG_OK;
    (void)hipStreamSynchronize(n->stream);
    free_grid(n);
    void* p[] = {n->w, n->grad, n->m, n->v, n->scal, n->rpart, n->ticket, n->zeros, n->sink};
    for (void* q : p)
        if (q) (void)hipFree(q);
    for (int l = 0; l < NL; ++l) {
        if (n->wf[l]) (void)hipFree(n->wf[l]);
        if (n->wb[l]) (void)hipFree(n->wb[l]);
    }
    delete n;
    return PCG_OK;
}

int cnn_num_weights(void) { return NW; }

pcg_status cnn_set_weights(cnn_net n, const float* w_dev) {
    if (!n || !w_dev) return err(PCG_E_ARG, "cnn_set_weights: null argument");
    CHK(hipMemcpyAsync(n->w, w_dev, sizeof(float) * NW, hipMemcpyDeviceToDevice, n->stream));
    CHK(hipMemsetAsync(n->m, 0, sizeof(float) * NW, n->stream));
    CHK(hipMemsetAsync(n->v, 0, sizeof(float) * NW, n->stream));
    n->step = 0;
    n->dirty = true;
    return PCG_OK;
}

pcg_status cnn_get_weights(cnn_net n, float* w_dev) {
    if (!n || !w_dev) return err(PCG_E_ARG, "cnn_get_weights: null argument");
    CHK(hipMemcpyAsync(w_dev, n->w, sizeof(float) * NW, hipMemcpyDeviceToDevice, n->stream));
    return PCG_OK;
}

pcg_status cnn_get_adam(cnn_net n, float* m_dev, float* v_dev, int64_t* step) {
    if (!n || !m_dev || !v_dev) return err(PCG_E_ARG, "cnn_get_adam: null argument");
    CHK(hipMemcpyAsync(m_dev, n->m, sizeof(float) * NW, hipMemcpyDeviceToDevice, n->stream));
    CHK(hipMemcpyAsync(v_dev, n->v, sizeof(float) * NW, hipMemcpyDeviceToDevice, n->stream));
    if (step) *step = n->step;
    return PCG_OK;
}

pcg_status cnn_set_adam(cnn_net n, const float* m_dev, const float* v_dev, int64_t step) {
    if (!n || !m_dev || !v_dev) return err(PCG_E_ARG, "cnn_set_adam: null argument");
    if (step < 0 || step > INT32_MAX) return err(PCG_E_ARG, "cnn_set_adam: step %lld out of range", (long long)step);
    CHK(hipMemcpyAsync(n->m, m_dev, sizeof(float) * NW, hipMemcpyDeviceToDevice, n->stream));
    CHK(hipMemcpyAsync(n->v, v_dev, sizeof(float) * NW, hipMemcpyDeviceToDevice, n->stream));
    n->step = (int)step;
    return PCG_OK;
}

pcg_status cnn_forward(cnn_net n, int nx, int ny, int nz, pcg_dtype rdt, const void* r, const float* g,
                       const double* rr_dev, float* z) {
    if (!n || !r || !z) return err(PCG_E_ARG, "cnn_forward: null argument");
    if (nx < 1 || ny < 1 || nz < 1) return err(PCG_E_ARG, "cnn_forward: bad dims");
    if (rdt != PCG_F32 && rdt != PCG_F64 && rdt != PCG_BF16)
        return err(PCG_E_UNSUPPORTED, "cnn_forward: r must be F32, F64 or BF16");
    pcg_status st = ensure_grid(n, nx, ny, nz);
    if (st != PCG_OK) return st;
    st = ensure_swizzled(n);
    if (st != PCG_OK) return st;
    // layer 1 packs its input from r and g itself (no pass through in0)
    CHK(launch_conv3d_input(n->nx, n->ny, n->nz, rdt, r, g, rr_dev, n->wf[0], n->h1, n->zeros, n->sink, n->stream));
    return forward(n, z, rr_dev, rr_dev ? 1.0 / std::sqrt((double)n->nvox) : 1.0, true);
}

pcg_status cnn_loss_grad(cnn_net n, int nx, int ny, int nz, const void* pairs, const float* g, int batch,
                         float* grad_dev, double* loss_dev) {
    Range range("cnn_loss_grad");
    if (!n || !pairs || batch < 1) return err(PCG_E_ARG, "cnn_loss_grad: bad argument");
    if (n->op && !ctx_is_f32_grid(n->op, nx, ny, nz))
        return err(PCG_E_ARG, "cnn_loss_grad: the operator's context is not an F32 context on this grid");
    pcg_status st = ensure_grid(n, nx, ny, nz);
    if (st != PCG_OK) return st;
    st = ensure_swizzled(n);
    if (st != PCG_OK) return st;
    hipStream_t s = n->stream;
    const int64_t nv = n->nvox;
    const float inv_b = 1.f / (float)batch;
    float* G = grad_dev ? grad_dev : n->grad;
    CHK(hipMemsetAsync(n->scal, 0, 4 * sizeof(double), s));
    Red red{n->rpart, n->ticket, (size_t)2 * DOT_MAX_BLOCKS};
    for (int b = 0; b < batch; ++b) {
        const uint16_t* rh = static_cast<const uint16_t*>(pairs) + (size_t)(2 * b) * nv;
        const uint16_t* eh = rh + nv;
        CHK(launch_pack_input(PCG_BF16, nv, rh, g, nullptr, n->in0, s));
        st = forward(n, n->out, nullptr, 1.0);
        if (st != PCG_OK) return st;
        if (n->op) {
            const float* dinv = ctx_dinv_f32(n->op);
            CHK(launch_anorm_u(nv, n->out, rh, dinv, n->u, s));
            CHK(ctx_apply_f32(n->op, n->u, n->au));
            CHK(launch_anorm_loss(nv, n->u, n->au, rh, n->energy, dinv, &n->scal[0], &n->scal[1], n->dout, n->dpack,
                                  red, s));
        } else {
            CHK(launch_loss(nv, n->out, eh, &n->scal[0], &n->scal[1], n->dout, n->dpack, red, s));
        }
        const bool acc = b > 0;
        const int X = nx, Y = ny, Z = nz;
        // layer 4: dW4 from (h3, dOut); dh3 = conv(dOut, mirrored W4) * (h3 > 0)
        CHK(launch_wgrad(X, Y, Z, 16, 1, n->h3, n->dout, true, n->zeros, n->partials, n->groups, s));
        CHK(launch_reduce_partials(n->partials, n->groups, 27 * 16, inv_b, acc, G + WOFF[3], s));
        CHK(launch_conv3d(X, Y, Z, 2, OUT_MASK, n->dpack, n->wb[3], n->da, n->h3, nullptr, 1.0, n->zeros, n->sink, s));
        // layer 3
        CHK(launch_wgrad(X, Y, Z, 16, 16, n->h2, n->da, false, n->zeros, n->partials, n->groups, s));
        CHK(launch_reduce_partials(n->partials, n->groups, 27 * 256, inv_b, acc, G + WOFF[2], s));
        CHK(launch_conv3d(X, Y, Z, 16, OUT_MASK, n->da, n->wb[2], n->db, n->h2, nullptr, 1.0, n->zeros, n->sink, s));
        // layer 2
        CHK(launch_wgrad(X, Y, Z, 16, 16, n->h1, n->db, false, n->zeros, n->partials, n->groups, s));
        CHK(launch_reduce_partials(n->partials, n->groups, 27 * 256, inv_b, acc, G + WOFF[1], s));
        CHK(launch_conv3d(X, Y, Z, 16, OUT_MASK, n->db, n->wb[1], n->da, n->h1, nullptr, 1.0, n->zeros, n->sink, s));
        // layer 1
        CHK(launch_wgrad(X, Y, Z, 2, 16, n->in0, n->da, false, n->zeros, n->partials, n->groups, s));
        CHK(launch_reduce_partials(n->partials, n->groups, 27 * 32, inv_b, acc, G + WOFF[0], s));
    }
    if (loss_dev) {
        // mean loss over the batch
        double h[4];
        CHK(hipMemcpyAsync(h, n->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        CHK(hipStreamSynchronize(s));
        const double mean = h[0] / batch;
        CHK(hipMemcpyAsync(loss_dev, &mean, sizeof(double), hipMemcpyHostToDevice, s));
        CHK(hipStreamSynchronize(s));
    }
    return PCG_OK;
}

pcg_status cnn_set_operator(cnn_net n, pcg_ctx ctx) {
    if (!n) return err(PCG_E_ARG, "cnn_set_operator: null network");
    if (ctx && ctx_stream(ctx) != n->stream)
        return err(PCG_E_ARG, "cnn_set_operator: the network and the context must use the same stream");
    n->op = ctx;
    return PCG_OK;
}

pcg_status cnn_set_loss_norm(cnn_net n, int mode) {
    if (!n) return err(PCG_E_ARG, "cnn_set_loss_norm: null network");
    if (mode != 0 && mode != 1) return err(PCG_E_ARG, "cnn_set_loss_norm: mode must be 0 or 1 (got %d)", mode);
    n->energy = mode == 1;
    return PCG_OK;
}

pcg_status cnn_adam_step(cnn_net n, const float* grad_dev, float lr) {
    Range range("cnn_adam_step");
    if (!n) return err(PCG_E_ARG, "cnn_adam_step: null network");
    n->step += 1;
    CHK(launch_adam(NW, n->w, grad_dev ? grad_dev : n->grad, n->m, n->v, lr, n->step, n->stream));
    n->dirty = true;
    return PCG_OK;
}

pcg_status cnn_train_step(cnn_net n, int nx, int ny, int nz, const void* pairs, const float* g, int batch, float lr,
                          double* loss_dev) {
    Range range("cnn_train_step");
    pcg_status st = cnn_loss_grad(n, nx, ny, nz, pairs, g, batch, nullptr, loss_dev);
    if (st != PCG_OK) return st;
    return cnn_adam_step(n, nullptr, lr);
}

}  // extern "C"
