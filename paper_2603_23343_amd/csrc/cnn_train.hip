// cnn_train.hip -- training-step kernels of the learned preconditioner:
// relative-MSE and A-norm losses and their gradients, the weight gradient of a 3x3x3
// convolution on the matrix cores (rows split over work-groups, partials
// reduced in a fixed order, so the result is deterministic), and Adam
// (Kingma & Ba 2015) on FP32 master weights.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace pcgmi {

namespace {

__device__ __forceinline__ float bf16v(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }


// Weight gradient on the matrix cores. For tap t = (dz, dy, dx) and an
// output x-row (z, y):
//   dW[t][ci][co] += sum_x X[z+dz-1, y+dy-1, x+dx-1][ci] dY[z, y, x][co]
//                 = sum_x' X[z+dz-1, y+dy-1, x'][ci] dY[z, y, x'-(dx-1)][co],
// a 16 x 16 x K product (K = the row, 32 points per v_mfma_f32_16x16x32_bf16)
// with A = the neighbour row of X and B = the output row of dY shifted by
// the tap's x offset. A work-group stages, per chunk of up to WGM_K points
// of a row, the 9 neighbour rows of X and the 3 shifted copies of dY in LDS,
// transposed to [channel][x] (channels beyond CX / CY are zero); wave w
// accumulates all 27 taps over K-step w of every item in registers, and the
// four wavefronts' sums are added in a fixed order at the end. Rows are
// dealt to work-groups round-robin; partials[g][27][CX][CY] feed the
// fixed-order reduction, so the result is deterministic.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

constexpr int WGM_K = 128;           // points of a row per staged chunk
// LDS row pitch (bf16): 288 bytes. The products read 16 rows (one per lane
// of a 16-lane group) at this pitch; measured on MI355X, a 288-byte pitch
// serves such a ds_read_b128 without bank conflicts, 272 bytes (the former
// pitch) takes 1.6x as long, 256 bytes 5.9x.
constexpr int WGM_SP = WGM_K + 16;

// One voxel's channels as loaded: C = 16 BF16 channels (two 16-byte loads),
// C = 2 (one 4-byte load) or one FP32 channel (rounded to BF16 when staged).
// A voxel outside the grid or the chunk loads from a zeroed page instead, so
// the loads are unconditional and nothing is masked afterwards. word(i)
// holds channels 2i (low half) and 2i + 1 (high half).
template <int C, typename S> struct Vox;
template <> struct Vox<16, uint16_t> {
    static constexpr int WORDS = 8;
    uint4 a, b;
    __device__ __forceinline__ void load(const uint16_t* __restrict__ p, int64_t v, bool ok, const void* zeros) {
        const uint16_t* q = ok ? p + v * 16 : static_cast<const uint16_t*>(zeros);
        a = *reinterpret_cast<const uint4*>(q);
        b = *reinterpret_cast<const uint4*>(q + 8);
    }
    __device__ __forceinline__ uint32_t word(int i) const {
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        return w[i];
    }
};
template <> struct Vox<2, uint16_t> {
    static constexpr int WORDS = 1;
    uint32_t w;
    __device__ __forceinline__ void load(const uint16_t* __restrict__ p, int64_t v, bool ok, const void* zeros) {
        w = *reinterpret_cast<const uint32_t*>(ok ? p + v * 2 : static_cast<const uint16_t*>(zeros));
    }
    __device__ __forceinline__ uint32_t word(int) const { return w; }
};
template <> struct Vox<1, float> {
    static constexpr int WORDS = 1;
    float f;
    __device__ __forceinline__ void load(const float* __restrict__ p, int64_t v, bool ok, const void* zeros) {
        f = *(ok ? p + v : static_cast<const float*>(zeros));
    }
    __device__ __forceinline__ uint32_t word(int) const { return (uint32_t)f32_to_bf16_bits(f); }
};

// Stage points xp and xp + 1 of a row into the [channel][x] LDS layout: the
// 32-bit word at (channel c, xp) holds (c of point xp, c of point xp + 1).
// One byte permute per channel: from the words (2i, 2i + 1) of both points,
// selector 0x05040100 takes the low halves, 0x07060302 the high halves.
// Channels past the voxel's own stay zero (they were zeroed once).
template <class V>
__device__ __forceinline__ void stage_pair(uint16_t* __restrict__ lds_row0, const V& pa, const V& pb) {
#pragma unroll
    for (int i = 0; i < V::WORDS; ++i) {
        const uint32_t wa = pa.word(i), wb = pb.word(i);
        *reinterpret_cast<uint32_t*>(lds_row0 + (2 * i) * WGM_SP) = __builtin_amdgcn_perm(wb, wa, 0x05040100u);
        *reinterpret_cast<uint32_t*>(lds_row0 + (2 * i + 1) * WGM_SP) = __builtin_amdgcn_perm(wb, wa, 0x07060302u);
    }
}

// A staged chunk: a row (y, z) of the output and points [x0, x0 + len).
struct WgItem {
    int y, z, row, x0, len, kp;  // kp: len rounded up to 32 (the products' K)
};

// Rows staged per item: the 9 neighbour rows of X (q = 3 dz + dy) and the 3
// shifted copies of dY (q = 9 + shift), 64 point pairs each: wavefront w
// stages rows q = w, w + 4, w + 8, every lane the same pair column.
template <int CX, int CY, typename Y>
__global__ void __launch_bounds__(256, 2) k_wgrad_mfma(int nx, int ny, int nz, const uint16_t* __restrict__ X,
                                                    const Y* __restrict__ dY, const void* __restrict__ zeros,
                                                    float* __restrict__ partials) {
    static_assert(WGM_K == 128, "one pair column per lane");
    __shared__ __attribute__((aligned(16))) uint16_t lds[12 * 16 * WGM_SP];
    uint16_t* const xs = lds;                    // the 9 neighbour rows of X
    uint16_t* const ys = lds + 9 * 16 * WGM_SP;  // the 3 shifted rows of dY
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, kg = lane >> 4;
    const int xp = 2 * lane;  // this lane's pair column
    f32x4_t acc[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int nch = (nx + WGM_K - 1) / WGM_K;
    const int nitems = ny * nz * nch;
    // XCD-aware dealing: work-group b runs on XCD b mod 8; with a grid that is
    // a multiple of 8, each XCD takes a contiguous slab of rows, so the
    // neighbour rows a work-group stages are mostly in its XCD's L2.
    int first = blockIdx.x, last = nitems, step = gridDim.x;
    if (gridDim.x % 8 == 0) {
        const int xcd = blockIdx.x % 8, per = gridDim.x / 8;
        first = (int)((int64_t)nitems * xcd / 8) + (int)(blockIdx.x / 8);
        last = (int)((int64_t)nitems * (xcd + 1) / 8);
        step = per;
    }
    auto geom = [&](int item) {
        WgItem it;
        const int ch = item % nch;
        it.row = item / nch;
        it.y = it.row % ny;
        it.z = it.row / ny;
        it.x0 = ch * WGM_K;
        it.len = min(WGM_K, nx - it.x0);
        it.kp = (it.len + 31) & ~31;
        return it;
    };
    // The next item's points are loaded into registers while the current
    // item's products run; a loop that stored each piece into LDS before
    // loading the next waited for every load in turn.
    Vox<CX, uint16_t> xa[3], xb[3];
    Vox<CY, Y> ya, yb;
    // Every load is issued on every path (a slot a wavefront does not use
    // reads the zero page): loads under branches kept these registers in
    // scratch memory.
    auto fetch = [&](const WgItem& it) {
        const bool pa = xp < it.len, pb = xp + 1 < it.len;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int q = wu + 4 * j;  // wave-uniform; rows q < 9 are X rows
            const int qx = q < 9 ? q : 0;
            const int zz = it.z + qx / 3 - 1, yy = it.y + qx % 3 - 1;
            const bool rok = q < 9 && zz >= 0 && zz < nz && yy >= 0 && yy < ny;
            const int64_t base = ((int64_t)zz * ny + yy) * nx + it.x0 + xp;
            xa[j].load(X, base, rok && pa, zeros);
            xb[j].load(X, base + 1, rok && pb, zeros);
        }
        // the dY row of wavefronts 1-3 (their third row q = 9 + shift)
        const int sft = wu - 1;
        const int ca = it.x0 + xp - (sft - 1);  // dY column feeding x' = x0 + xp (+1)
        const int64_t base = (int64_t)it.row * nx + ca;
        ya.load(dY, base, wu > 0 && pa && ca >= 0 && ca < nx, zeros);
        yb.load(dY, base + 1, wu > 0 && pb && ca + 1 >= 0 && ca + 1 < nx, zeros);
    };
    // LDS: [row or shift][channel][x], transposed from the voxel-major input.
    auto stage = [&]() {
        stage_pair(&xs[(wu * 16) * WGM_SP + xp], xa[0], xb[0]);
        stage_pair(&xs[((wu + 4) * 16) * WGM_SP + xp], xa[1], xb[1]);
        if (wu == 0) stage_pair(&xs[(8 * 16) * WGM_SP + xp], xa[2], xb[2]);
        else stage_pair(&ys[((wu - 1) * 16) * WGM_SP + xp], ya, yb);
    };
    // Channels a narrow input never writes (CX = 2, CY = 1) stay zero.
    if constexpr (CX < 16 || CY < 16) {
        for (int i = tid; i < 9 * 16 * WGM_SP / 2; i += 256) reinterpret_cast<uint32_t*>(xs)[i] = 0u;
        for (int i = tid; i < 3 * 16 * WGM_SP / 2; i += 256) reinterpret_cast<uint32_t*>(ys)[i] = 0u;
    }
    // Wavefront w takes K-step w (points 32 w .. + 31) of every item for all
    // 27 taps: 9 X fragments and 3 dY fragments feed 27 products, each
    // fragment read once per work-group. (Taps dealt to wavefronts, each
    // wavefront running every K-step, read each X fragment three times and
    // measured 1.15x slower per 16 -> 16 layer.)
    auto products = [&](int kp) {
        const int kb = 32 * wu;
        if (kb >= kp) return;
        const int ko = kb + 8 * kg;
        bf16x8_t b[3];
#pragma unroll
        for (int sft = 0; sft < 3; ++sft)
            b[sft] = *reinterpret_cast<const bf16x8_t*>(&ys[(sft * 16 + m) * WGM_SP + ko]);
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&xs[(r * 16 + m) * WGM_SP + ko]);
#pragma unroll
            for (int sft = 0; sft < 3; ++sft)
                acc[3 * r + sft] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[sft], acc[3 * r + sft], 0, 0, 0);
        }
    };
    WgItem cur{};
    if (first < last) {
        cur = geom(first);
        fetch(cur);
    }
    for (int item = first; item < last; item += step) {
        __syncthreads();  // the previous item's fragments have been read
        stage();
        __syncthreads();
        const int kp = cur.kp;
        if (item + step < last) {
            cur = geom(item + step);
            fetch(cur);
        }
        products(kp);
    }
    // Sum the four wavefronts' accumulators in a fixed order through LDS
    // (the staging area holds two wavefronts' 27 x 64 x 4 floats): waves 2, 3
    // hand theirs to 0, 1, then wave 1 to wave 0.
    float* red = reinterpret_cast<float*>(lds);
    static_assert(sizeof(lds) >= 2 * 27 * 64 * 4 * sizeof(float), "reduction area");
    __syncthreads();
    if (wu >= 2) {
#pragma unroll
        for (int t = 0; t < 27; ++t)
            *reinterpret_cast<f32x4_t*>(&red[(((wu - 2) * 27 + t) * 64 + lane) * 4]) = acc[t];
    }
    __syncthreads();
    if (wu < 2) {
#pragma unroll
        for (int t = 0; t < 27; ++t) acc[t] += *reinterpret_cast<const f32x4_t*>(&red[((wu * 27 + t) * 64 + lane) * 4]);
    }
    __syncthreads();
    if (wu == 1) {
#pragma unroll
        for (int t = 0; t < 27; ++t) *reinterpret_cast<f32x4_t*>(&red[(t * 64 + lane) * 4]) = acc[t];
    }
    __syncthreads();
    if (wu != 0) return;
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] += *reinterpret_cast<const f32x4_t*>(&red[(t * 64 + lane) * 4]);
    // lane holds C[ci = 4 kg + i][co = m] of every tap
    float* out = partials + (size_t)blockIdx.x * 27 * CX * CY;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ci = 4 * kg + i;
            if (ci < CX && m < CY) out[(t * CX + ci) * CY + m] = acc[t][i];
        }
    }
}

// grad[j] (+)= scale * sum_g partials[g][j]. A work-group owns 64 outputs;
// thread (q, j) with q = tid / 64 < RP_WAVES sums groups q, q + RP_WAVES,
// ... for output j in FP64 (four independent loads in flight), and the
// RP_WAVES sums are added pairwise in a fixed tree, so the result does not
// depend on timing.
constexpr int RP_WAVES = 16;
__global__ void __launch_bounds__(64 * RP_WAVES) k_reduce_partials(const float* __restrict__ partials, int ngroups,
                                                                   int len, float scale, int accumulate,
                                                                   float* __restrict__ grad) {
    __shared__ double part[RP_WAVES][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < len) {
        int g = q;
        for (; g + 3 * RP_WAVES < ngroups; g += 4 * RP_WAVES) {
#pragma unroll
            for (int u = 0; u < 4; ++u) s[u] += (double)partials[(size_t)(g + u * RP_WAVES) * len + j];
        }
        for (; g < ngroups; g += RP_WAVES) s[0] += (double)partials[(size_t)g * len + j];
    }
    part[q][lane] = (s[0] + s[1]) + (s[2] + s[3]);
    __syncthreads();
#pragma unroll
    for (int w = RP_WAVES / 2; w >= 1; w /= 2) {
        if (q < w) part[q][lane] += part[q + w][lane];
        __syncthreads();
    }
    if (q == 0 && j < len) {
        const float v = (float)(part[0][lane] * (double)scale);
        grad[j] = accumulate ? grad[j] + v : v;
    }
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
    double v[2] = {a, b};
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        red.partials[2 * blockIdx.x] = v[0];
        red.partials[2 * blockIdx.x + 1] = v[1];
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

// A-norm loss of one sample in the Jacobi-plus-correction form. With the
// network output N (FP32), the pair (rh, eh) (bf16) and the Jacobi scale
// dinv (null: the constant 1/6):
//   u = N + dinv rh - eh                          (k_anorm_u)
//   L = u.Au / (rh.dinv rh),  dL/dN = 2 Au / (rh.dinv rh)
// k_anorm_sums reduces u.Au and the normaliser into loss_acc and coef: rh.dinv rh,
// or (eh given) rh.eh, the error's energy e.Ae when rh = A eh.
__global__ void __launch_bounds__(256) k_anorm_u(int64_t n, const float* __restrict__ out,
                                                 const uint16_t* __restrict__ rh, const uint16_t* __restrict__ eh,
                                                 const float* __restrict__ dinv, float* __restrict__ u) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float d = dinv ? dinv[i] : (1.f / 6.f);
        u[i] = out[i] + d * bf16v(rh[i]) - bf16v(eh[i]);
    }
}

__global__ void __launch_bounds__(256) k_anorm_sums(int64_t n, const float* __restrict__ u,
                                                    const float* __restrict__ au, const uint16_t* __restrict__ rh,
                                                    const uint16_t* __restrict__ eh, const float* __restrict__ dinv,
                                                    double* loss_acc, double* coef, Red red) {
    __shared__ double scratch[32];
    const int64_t stride = (int64_t)gridDim.x * 256;
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const double r = (double)bf16v(rh[i]);
        a += (double)u[i] * (double)au[i];
        b += eh ? r * (double)bf16v(eh[i]) : (dinv ? (double)dinv[i] : 1.0 / 6.0) * r * r;
    }
    double v[2] = {a, b};
    block_reduce<2, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        red.partials[2 * blockIdx.x] = v[0];
        red.partials[2 * blockIdx.x + 1] = v[1];
    }
}

// One work-group: the loss sums' partials in index order -> loss_acc +=
// tot0 / tot1 and coef = 2 / tot1 (a kernel boundary instead of an
// agent-scope release fence per work-group of the sums).
__global__ void __launch_bounds__(256) k_loss_finish(const double* __restrict__ partials, unsigned nblocks,
                                                     double* loss_acc, double* coef) {
    __shared__ double lds[32];
    double acc[2] = {0.0, 0.0};
    for (unsigned i = threadIdx.x; i < nblocks; i += 256) {
        acc[0] += partials[2 * i];
        acc[1] += partials[2 * i + 1];
    }
    block_reduce<2, 0u>(acc, lds);
    if (threadIdx.x == 0) {
        *loss_acc += acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
        *coef = acc[1] > 0.0 ? 2.0 / acc[1] : 0.0;
    }
}

// dOut = coef Au: FP32 for the weight gradient, packed (bf16, 0) for dgrad.
__global__ void __launch_bounds__(256) k_scale_grad(int64_t n, const float* __restrict__ au, const double* coef,
                                                    float* __restrict__ dout, uint32_t* __restrict__ dpack) {
    const float c = (float)*coef;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float g = c * au[i];
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

// Work-groups of the weight-gradient launch (and partial sets to reduce):
// one per staged row chunk up to 512 (two per CU, as the LDS allows); a
// multiple of 8 from 64 rows on, for the XCD slabs.
int wgrad_groups(int nx, int ny, int nz) {
    const int64_t items = (int64_t)ny * nz * ((nx + WGM_K - 1) / WGM_K);
    if (items < 64) return (int)(items < 1 ? 1 : items);
    const int64_t g = items > 512 ? 512 : items;  // two 55 KB-LDS work-groups per CU
    return (int)(g / 8 * 8);
}

// zeros: a device buffer of at least 32 zero bytes (read in place of
// points outside the grid).
hipError_t launch_wgrad(int nx, int ny, int nz, int cx, int cy, const void* X, const void* dY, bool dy_f32,
                        const void* zeros, float* partials, int groups, hipStream_t s) {
    auto x16 = static_cast<const uint16_t*>(X);
    if (cx == 16 && cy == 16 && !dy_f32)
        hipLaunchKernelGGL((k_wgrad_mfma<16, 16, uint16_t>), dim3(groups), dim3(256), 0, s, nx, ny, nz, x16,
                           static_cast<const uint16_t*>(dY), zeros, partials);
    else if (cx == 2 && cy == 16 && !dy_f32)
        hipLaunchKernelGGL((k_wgrad_mfma<2, 16, uint16_t>), dim3(groups), dim3(256), 0, s, nx, ny, nz, x16,
                           static_cast<const uint16_t*>(dY), zeros, partials);
    else if (cx == 16 && cy == 1 && dy_f32)
        hipLaunchKernelGGL((k_wgrad_mfma<16, 1, float>), dim3(groups), dim3(256), 0, s, nx, ny, nz, x16,
                           static_cast<const float*>(dY), zeros, partials);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* partials, int groups, int len, float scale, bool accumulate,
                                  float* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3((len + 63) / 64), dim3(64 * RP_WAVES), 0, s, partials, groups, len, scale,
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
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, red.partials, (unsigned)nb, loss_acc, coef);
    hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)nb), dim3(256), 0, s, n, out, t16, coef, dout,
                       static_cast<uint32_t*>(dpack));
    return hipGetLastError();
}

hipError_t launch_anorm_u(int64_t n, const float* out, const void* pair, const float* dinv, float* u,
                          hipStream_t s) {
    int64_t nb = (n + 1023) / 1024;
    nb = nb < 1 ? 1 : (nb > 8192 ? 8192 : nb);
    auto rh = static_cast<const uint16_t*>(pair);
    hipLaunchKernelGGL(k_anorm_u, dim3((unsigned)nb), dim3(256), 0, s, n, out, rh, rh + n, dinv, u);
    return hipGetLastError();
}

hipError_t launch_anorm_loss(int64_t n, const float* u, const float* au, const void* rh, bool energy,
                             const float* dinv, double* loss_acc, double* coef, float* dout, void* dpack, Red red,
                             hipStream_t s) {
    int64_t nb = (n + 1023) / 1024;
    nb = nb < 1 ? 1 : (nb > DOT_MAX_BLOCKS ? DOT_MAX_BLOCKS : nb);
    if ((size_t)2 * nb > red.cap) return hipErrorInvalidValue;
    auto r16 = static_cast<const uint16_t*>(rh);
    hipLaunchKernelGGL(k_anorm_sums, dim3((unsigned)nb), dim3(256), 0, s, n, u, au, r16, energy ? r16 + n : nullptr,
                       dinv, loss_acc, coef, red);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, red.partials, (unsigned)nb, loss_acc, coef);
    hipLaunchKernelGGL(k_scale_grad, dim3((unsigned)nb), dim3(256), 0, s, n, au, coef, dout,
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
