// cnn_train.hip -- training-step kernels of the learned preconditioner:
// relative-MSE loss and its gradient, the weight gradient of a 3x3x3
// convolution (split over voxels with a fixed-order reduction, so the result
// is deterministic), and Adam (Kingma & Ba 2015) on FP32 master weights.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace pcgmi {

namespace {

__device__ __forceinline__ float bf16v(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

template <typename Y> __device__ __forceinline__ float ld_val(const Y* p, int64_t i);
template <> __device__ __forceinline__ float ld_val<uint16_t>(const uint16_t* p, int64_t i) { return bf16v(p[i]); }
template <> __device__ __forceinline__ float ld_val<float>(const float* p, int64_t i) { return p[i]; }

// Weight gradient dW[t][cx][cy] = sum_v X[v + off_t][cx] dY[v][cy] over a
// contiguous chunk of voxels per work-group; partials[g][27][CX][CY].
// Thread layout: pair = tid % (CX*CY), voxel lane = tid / (CX*CY).
template <int CX, int CY, typename Y>
__global__ void __launch_bounds__(256) k_wgrad(int nx, int ny, int nz, const uint16_t* __restrict__ X,
                                               const Y* __restrict__ dY, float* __restrict__ partials,
                                               int64_t chunk) {
    constexpr int NP = CX * CY, NV = 256 / NP;
    static_assert(256 % NP == 0, "pairs must divide the work-group");
    __shared__ float red[256];
    const int tid = threadIdx.x, pair = tid % NP, vl = tid / NP;
    const int cx = pair / CY, cy = pair % CY;
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t v0 = (int64_t)blockIdx.x * chunk, v1 = v0 + chunk < nvox ? v0 + chunk : nvox;
    float acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = 0.f;
    for (int64_t v = v0 + vl; v < v1; v += NV) {
        const float dy = ld_val<Y>(dY, v * CY + cy);
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int xx = x + (t % 3) - 1, yy = y + (t / 3) % 3 - 1, zz = z + t / 9 - 1;
            const bool in = xx >= 0 && xx < nx && yy >= 0 && yy < ny && zz >= 0 && zz < nz;
            const int64_t nb = in ? ((int64_t)zz * ny + yy) * nx + xx : 0;
            const float xv = bf16v(X[nb * CX + cx]);
            acc[t] += in ? xv * dy : 0.f;
        }
    }
    // Sum the NV voxel lanes of each pair in a fixed order.
    float* out = partials + (size_t)blockIdx.x * 27 * NP;
#pragma unroll 1
    for (int t = 0; t < 27; ++t) {
        red[tid] = acc[t];
        __syncthreads();
        if (vl == 0) {
            float s = 0.f;
            for (int q = 0; q < NV; ++q) s += red[q * NP + pair];
            out[t * NP + pair] = s;
        }
        __syncthreads();
    }
}

// grad[j] (+)= scale * sum_g partials[g][j], g in index order.
__global__ void k_reduce_partials(const float* __restrict__ partials, int ngroups, int len, float scale,
                                  int accumulate, float* __restrict__ grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += (double)partials[(size_t)g * len + j];
    const float v = (float)(s * (double)scale);
    grad[j] = accumulate ? grad[j] + v : v;
}

// Loss of one sample: out (FP32 network output) against the target channel of
// a pair (bf16, stride 1); totals {sum (o - t)^2, sum t^2} -> loss_acc += L,
// coef = 2 / sum t^2 for the gradient pass.
__global__ void __launch_bounds__(256) k_loss_sums(int64_t n, const float* __restrict__ out,
                                                   const uint16_t* __restrict__ tgt, double* loss_acc,
                                                   double* coef, Red red) {
    __shared__ double scratch[32];
    const int64_t stride = (int64_t)gridDim.x * 256;
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const double t = (double)bf16v(tgt[i]);
        const double dlt = (double)out[i] - t;
        a += dlt * dlt;
        b += t * t;
    }
    double v[2] = {a, b}, tot[2];
    if (grid_reduce<2, 0u>(v, red.partials, red.ticket, gridDim.x, blockIdx.x, scratch, tot) && threadIdx.x == 0) {
        *loss_acc += tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
        *coef = tot[1] > 0.0 ? 2.0 / tot[1] : 0.0;
    }
}

// dOut = coef (o - t): FP32 for the weight gradient and packed (bf16, 0) for
// the input-gradient convolution.
__global__ void __launch_bounds__(256) k_loss_grad(int64_t n, const float* __restrict__ out,
                                                   const uint16_t* __restrict__ tgt, const double* coef,
                                                   float* __restrict__ dout, uint32_t* __restrict__ dpack) {
    const float c = (float)*coef;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float g = c * (out[i] - bf16v(tgt[i]));
        dout[i] = g;
        dpack[i] = (uint32_t)f32_to_bf16_bits(g);
    }
}

__global__ void k_adam(int n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// One training pair from a solver snapshot: rho = rms(r) from the device
// scalar rr; out[0..n) = bf16(r / rho), out[n..2n) = bf16((x* - x) / rho).
__global__ void __launch_bounds__(256) k_make_pair(int64_t n, const double* __restrict__ r, const double* __restrict__ x,
                                                   const double* __restrict__ xs, const double* rr,
                                                   uint16_t* __restrict__ out) {
    const double inv = 1.0 / sqrt(*rr / (double)n);
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        out[i] = f32_to_bf16_bits((float)(r[i] * inv));
        out[n + i] = f32_to_bf16_bits((float)((xs[i] - x[i]) * inv));
    }
}

}  // namespace

hipError_t launch_make_pair(int64_t n, const double* r, const double* x, const double* xs, const double* rr,
                            void* out, hipStream_t s) {
    int64_t nb = (n + 1023) / 1024;
    nb = nb < 1 ? 1 : (nb > 8192 ? 8192 : nb);
    hipLaunchKernelGGL(k_make_pair, dim3((unsigned)nb), dim3(256), 0, s, n, r, x, xs, rr, static_cast<uint16_t*>(out));
    return hipGetLastError();
}

int wgrad_groups(int64_t nvox) {
    int64_t g = (nvox + 4095) / 4096;
    return (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

hipError_t launch_wgrad(int nx, int ny, int nz, int cx, int cy, const void* X, const void* dY, bool dy_f32,
                        float* partials, int groups, hipStream_t s) {
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int64_t chunk = (nvox + groups - 1) / groups;
    auto x16 = static_cast<const uint16_t*>(X);
    if (cx == 16 && cy == 16 && !dy_f32)
        hipLaunchKernelGGL((k_wgrad<16, 16, uint16_t>), dim3(groups), dim3(256), 0, s, nx, ny, nz, x16,
                           static_cast<const uint16_t*>(dY), partials, chunk);
    else if (cx == 2 && cy == 16 && !dy_f32)
        hipLaunchKernelGGL((k_wgrad<2, 16, uint16_t>), dim3(groups), dim3(256), 0, s, nx, ny, nz, x16,
                           static_cast<const uint16_t*>(dY), partials, chunk);
    else if (cx == 16 && cy == 1 && dy_f32)
        hipLaunchKernelGGL((k_wgrad<16, 1, float>), dim3(groups), dim3(256), 0, s, nx, ny, nz, x16,
                           static_cast<const float*>(dY), partials, chunk);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* partials, int groups, int len, float scale, bool accumulate,
                                  float* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((len + 255) / 256), dim3(256), 0, s, partials, groups, len, scale,
                       accumulate ? 1 : 0, grad);
    return hipGetLastError();
}

hipError_t launch_loss(int64_t n, const float* out, const void* tgt, double* loss_acc, double* coef, float* dout,
                       void* dpack, Red red, hipStream_t s) {
    int64_t nb = (n + 1023) / 1024;
    nb = nb < 1 ? 1 : (nb > DOT_MAX_BLOCKS ? DOT_MAX_BLOCKS : nb);
    if ((size_t)2 * nb > red.cap) return hipErrorInvalidValue;
    auto t16 = static_cast<const uint16_t*>(tgt);
    hipLaunchKernelGGL(k_loss_sums, dim3((unsigned)nb), dim3(256), 0, s, n, out, t16, loss_acc, coef, red);
    hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)nb), dim3(256), 0, s, n, out, t16, coef, dout,
                       static_cast<uint32_t*>(dpack));
    return hipGetLastError();
}

hipError_t launch_adam(int n, float* w, const float* g, float* m, float* v, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, n, w, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace pcgmi
