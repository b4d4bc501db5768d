// cnn.hip -- the learned preconditioner's network on gfx950: 3x3x3
// convolutions with zero padding as implicit GEMM on the matrix cores, plus
// the pieces of its training step.
//
// Layout. Activations are NDHWC: voxel-major [nz][ny][nx], channels
// innermost, BF16. A layer's FP32 master weight is W[27][Cin][Cout], tap
// t = 9 dz + 3 dy + dx (offsets -1..1). The network is 2 -> 16 -> 16 -> 16
// -> 1 with ReLU after the first three layers.
//
// Forward conv (implicit GEMM): M = voxels, N = Cout = 16, K = 27 * Cin.
// One v_mfma_f32_16x16x32_bf16 multiplies a 16 x 32 block of the patch
// matrix (16 voxels x 32 values of K) by a 32 x 16 block of the weights.
// Operand lane layout (lane l): A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l
// % 16] for j < 8, D[4 (l / 16) + i][l % 16] for i < 4. For Cin = 16 a K
// chunk covers two taps, so each lane's 8 A values are 8 consecutive
// channels of one neighbour: one 16-byte load. For Cin = 2 (the packed
// input) a chunk covers 16 taps and a lane gathers four (tap, 2-channel)
// pairs. Taps beyond 27 and neighbours outside the grid contribute zero.
// Weights are pre-swizzled into exactly the B lane layout, so each lane
// reads its 16 bytes per chunk with one load and keeps all chunks in
// registers. A work-group owns a 16 x 8 x 4 block of output voxels: it
// stages the block's input with its one-voxel halo (18 x 10 x 6 voxels) in
// LDS once, so every input voxel crosses L2 about twice instead of 27 times,
// and each wavefront computes 8 tiles of 16 voxels (x-rows of the block)
// from LDS. The 16 x 16 FP32 results go through LDS so each voxel's 16
// channels leave as two 16-byte stores.
//
// The transposed convolution of the backward pass (input gradient) is the
// same kernel with the taps mirrored and Cin/Cout swapped in the swizzle.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "internal.hpp"

namespace pcgmi {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

constexpr int CONV_WAVES = 4;     // wavefronts per work-group
constexpr int CONV_NT = 64 * CONV_WAVES;

__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }
__device__ __forceinline__ uint16_t bf16_bits(float f) { return f32_to_bf16_bits(f); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

struct Dims {
    int nx, ny, nz;
    int64_t nvox;
};

enum ConvOut : int {
    OUT_RELU_BF16 = 0,   // hidden layer: bf16(relu(D)), 16 channels
    OUT_SCALED_F32 = 1,  // last layer: out[v] = scale * D[v][0] (FP32, one channel)
    OUT_MASK_BF16 = 2,   // input gradient: bf16(D * (mask[v][c] > 0)), 16 channels
    OUT_LINEAR_BF16 = 3  // bf16(D), 16 channels
};

template <int CIN> struct ConvK {
    static constexpr int CHUNKS = CIN == 16 ? 14 : 2;  // 32-wide K chunks (27 taps padded)
};

// Output block per work-group and its input halo block.
constexpr int CB_X = 16, CB_Y = 8, CB_Z = 4;
constexpr int CH_X = CB_X + 2, CH_Y = CB_Y + 2, CH_Z = CB_Z + 2;
constexpr int CH_VOX = CH_X * CH_Y * CH_Z;
constexpr int CB_ROWS = CB_Y * CB_Z;                 // 16-voxel x-rows (tiles) per block
constexpr int CB_TILES = CB_ROWS / CONV_WAVES;       // tiles per wavefront

// in: [nvox][CIN] bf16 bits. wsw: [CHUNKS][64 lanes][8] bf16 bits (B operand).
template <int CIN, int MODE>
__global__ void __launch_bounds__(CONV_NT) k_conv3d(Dims d, int nbx, int nby, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                    const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                    double scale_mul) {
    constexpr int NCH = ConvK<CIN>::CHUNKS;
    constexpr int VB = CIN * 2;  // bytes per staged voxel (32 or 4)
    __shared__ __attribute__((aligned(16))) unsigned char halo[CH_VOX * VB];
    __shared__ float lds_d[CONV_WAVES][16][17];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
    const int x0 = bx * CB_X, y0 = by * CB_Y, z0 = bz * CB_Z;

    // Stage the halo block (zero outside the grid).
    if constexpr (CIN == 16) {
        for (int it = tid; it < CH_VOX * 2; it += CONV_NT) {
            const int h = it >> 1, half = it & 1;
            const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
                v = *reinterpret_cast<const uint4*>(in + (((int64_t)gz * d.ny + gy) * d.nx + gx) * 16 + 8 * half);
            *reinterpret_cast<uint4*>(halo + (size_t)it * 16) = v;
        }
    } else {
        for (int h = tid; h < CH_VOX; h += CONV_NT) {
            const int hx = h % CH_X, hy = (h / CH_X) % CH_Y, hz = h / (CH_X * CH_Y);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint32_t v = 0u;
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
                v = *reinterpret_cast<const uint32_t*>(in + (((int64_t)gz * d.ny + gy) * d.nx + gx) * 2);
            *reinterpret_cast<uint32_t*>(halo + (size_t)h * 4) = v;
        }
    }

    // B operands: all weight chunks in registers.
    bf16x8_t bw[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const uint16_t* p = wsw + ((size_t)c * 64 + lane) * 8;
        Vec16<bf16> raw = *reinterpret_cast<const Vec16<bf16>*>(p);
#pragma unroll
        for (int j = 0; j < 8; ++j) bw[c][j] = bits_to_bf16(raw.e[j].bits);
    }
    __syncthreads();

    const int row = lane & 15, kgrp = lane >> 4;  // A: voxel row (x within the tile), K group of 8
    f32x4_t acc[CB_TILES];
#pragma unroll
    for (int tt = 0; tt < CB_TILES; ++tt) acc[tt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
        for (int tt = 0; tt < CB_TILES; ++tt) {
            const int q = wid + CONV_WAVES * tt;  // tile row in the block
            const int yl = q % CB_Y, zl = q / CB_Y;
            bf16x8_t a;
            if constexpr (CIN == 16) {
                const int tap = 2 * c + (kgrp >> 1);
                const int tq = tap < 27 ? tap : 0;
                const int h = ((zl + tq / 9) * CH_Y + (yl + (tq / 3) % 3)) * CH_X + row + tq % 3;
                const uint4 raw = *reinterpret_cast<const uint4*>(halo + (size_t)h * 32 + 16 * (kgrp & 1));
                const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t v = tap < 27 ? w[j] : 0u;
                    a[2 * j] = bits_to_bf16((uint16_t)(v & 0xffffu));
                    a[2 * j + 1] = bits_to_bf16((uint16_t)(v >> 16));
                }
            } else {
                // k = 2 tap + channel; lane's 8 values: taps 16 c + 4 kgrp + (0..3), 2 channels each
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const int tap = 16 * c + 4 * kgrp + qq;
                    const int tq = tap < 27 ? tap : 0;
                    const int h = ((zl + tq / 9) * CH_Y + (yl + (tq / 3) % 3)) * CH_X + row + tq % 3;
                    const uint32_t w2 = *reinterpret_cast<const uint32_t*>(halo + (size_t)h * 4);
                    const uint32_t v = tap < 27 ? w2 : 0u;
                    a[2 * qq] = bits_to_bf16((uint16_t)(v & 0xffffu));
                    a[2 * qq + 1] = bits_to_bf16((uint16_t)(v >> 16));
                }
            }
            acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[c], acc[tt], 0, 0, 0);
        }
    }

    // Results: lane holds D[4 kgrp + i][row] (voxel 4 kgrp + i of the tile, channel row).
    float scale = 0.f;
    if constexpr (MODE == OUT_SCALED_F32) scale = (float)(scale_rms2 ? sqrt(*scale_rms2) * scale_mul : scale_mul);
#pragma unroll
    for (int tt = 0; tt < CB_TILES; ++tt) {
        const int q = wid + CONV_WAVES * tt;
        const int gy = y0 + q % CB_Y, gz = z0 + q / CB_Y;
        const bool rok = gy < d.ny && gz < d.nz;
        const int64_t vrow = ((int64_t)gz * d.ny + gy) * d.nx;
        if constexpr (MODE == OUT_SCALED_F32) {
            if (row == 0 && rok) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int gx = x0 + 4 * kgrp + i;
                    if (gx < d.nx) static_cast<float*>(out)[vrow + gx] = scale * acc[tt][i];
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) lds_d[wid][4 * kgrp + i][row] = acc[tt][i];
            // wavefront-scope LDS hand-off (this wavefront's lanes read what its other lanes wrote)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // lanes 0..31 write the tile's 16 voxels x 16 channels as 8-channel (16-byte) pieces.
            if (lane < 32) {
                const int vi = lane >> 1, c0 = 8 * (lane & 1);
                const int gx = x0 + vi;
                if (rok && gx < d.nx) {
                    const int64_t v = vrow + gx;
                    Vec16<bf16> o;
                    Vec16<bf16> m;
                    if constexpr (MODE == OUT_MASK_BF16) m = *reinterpret_cast<const Vec16<bf16>*>(mask + v * 16 + c0);
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        float val = lds_d[wid][vi][c0 + j];
                        if constexpr (MODE == OUT_RELU_BF16) val = val > 0.f ? val : 0.f;
                        if constexpr (MODE == OUT_MASK_BF16) val = bf16_val(m.e[j].bits) > 0.f ? val : 0.f;
                        o.e[j].bits = bf16_bits(val);
                    }
                    *reinterpret_cast<Vec16<bf16>*>(static_cast<uint16_t*>(out) + v * 16 + c0) = o;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Network input: in[v] = (bf16(r[v] / rms), bf16(g[v])), rms = sqrt(rr / nvox)
// from a device scalar ||r||^2 (rr) or, when rr is null, in[v] = (bf16(r[v]), bf16(g[v])).
template <typename T>
__global__ void __launch_bounds__(256) k_pack_input(int64_t n, const T* __restrict__ r, const float* __restrict__ g,
                                                    const double* rr, uint32_t* __restrict__ out) {
    const float inv = rr ? (float)(1.0 / sqrt(*rr / (double)n)) : 1.f;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float a = (float)to_c(r[i]) * inv;
        const float b = g ? g[i] : 0.f;
        out[i] = (uint32_t)bf16_bits(a) | ((uint32_t)bf16_bits(b) << 16);
    }
}

// Swizzle FP32 master weights W[27][cin][cout] into the B-operand lane
// layout of k_conv3d for input width CIN (2 or 16; cin <= CIN, cout <= 16,
// missing entries zero). mirror: use W[26 - t][co][ci] (input gradient:
// mirrored taps, input and output channels swapped).
__global__ void k_swizzle_weights(const float* __restrict__ w, int cin, int cout, int CIN, int mirror,
                                  uint16_t* __restrict__ out) {
    const int nch = CIN == 16 ? 14 : 2;
    const int total = nch * 64 * 8;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int j = idx % 8, lane = (idx / 8) % 64, c = idx / 512;
        const int n = lane & 15, k = 8 * (lane >> 4) + j;  // B[k][n]
        int tap, ci;
        if (CIN == 16) {
            tap = 2 * c + k / 16;
            ci = k % 16;
        } else {
            tap = 16 * c + k / 2;
            ci = k % 2;
        }
        float v = 0.f;
        // effective layer: input channels = ci (< cin_eff), output channels = n (< cout_eff)
        const int cin_eff = mirror ? cout : cin, cout_eff = mirror ? cin : cout;
        if (tap < 27 && ci < cin_eff && n < cout_eff) {
            if (mirror) v = w[((size_t)(26 - tap) * cin + n) * cout + ci];
            else v = w[((size_t)tap * cin + ci) * cout + n];
        }
        out[idx] = bf16_bits(v);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

hipError_t launch_conv3d(int nx, int ny, int nz, int cin, int mode, const void* in, const void* wsw, void* out,
                         const void* mask, const double* scale_rms2, double scale_mul, hipStream_t s) {
    Dims d{nx, ny, nz, (int64_t)nx * ny * nz};
    if (d.nvox == 0) return hipSuccess;
    const int nbx = (nx + CB_X - 1) / CB_X, nby = (ny + CB_Y - 1) / CB_Y, nbz = (nz + CB_Z - 1) / CB_Z;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    auto in16 = static_cast<const uint16_t*>(in);
    auto w16 = static_cast<const uint16_t*>(wsw);
    auto m16 = static_cast<const uint16_t*>(mask);
#define PCGMI_CONV(CI, MO) \
    hipLaunchKernelGGL((k_conv3d<CI, MO>), dim3((unsigned)nb), dim3(CONV_NT), 0, s, d, nbx, nby, in16, w16, out, m16, \
                       scale_rms2, scale_mul)
    if (cin == 16) {
        switch (mode) {
            case OUT_RELU_BF16: PCGMI_CONV(16, OUT_RELU_BF16); break;
            case OUT_SCALED_F32: PCGMI_CONV(16, OUT_SCALED_F32); break;
            case OUT_MASK_BF16: PCGMI_CONV(16, OUT_MASK_BF16); break;
            case OUT_LINEAR_BF16: PCGMI_CONV(16, OUT_LINEAR_BF16); break;
            default: return hipErrorInvalidValue;
        }
    } else if (cin == 2) {
        switch (mode) {
            case OUT_RELU_BF16: PCGMI_CONV(2, OUT_RELU_BF16); break;
            case OUT_SCALED_F32: PCGMI_CONV(2, OUT_SCALED_F32); break;
            case OUT_MASK_BF16: PCGMI_CONV(2, OUT_MASK_BF16); break;
            case OUT_LINEAR_BF16: PCGMI_CONV(2, OUT_LINEAR_BF16); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef PCGMI_CONV
    return hipGetLastError();
}

hipError_t launch_pack_input(int dt, int64_t n, const void* r, const float* g, const double* rr, void* out,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 1023) / 1024;
    nb = nb > 8192 ? 8192 : nb;
    auto o = static_cast<uint32_t*>(out);
    if (dt == DT_F32)
        hipLaunchKernelGGL(k_pack_input<float>, dim3((unsigned)nb), dim3(256), 0, s, n, static_cast<const float*>(r), g, rr, o);
    else if (dt == DT_F64)
        hipLaunchKernelGGL(k_pack_input<double>, dim3((unsigned)nb), dim3(256), 0, s, n, static_cast<const double*>(r), g, rr, o);
    else if (dt == DT_BF16)
        hipLaunchKernelGGL(k_pack_input<bf16>, dim3((unsigned)nb), dim3(256), 0, s, n, static_cast<const bf16*>(r), g, rr, o);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_swizzle_weights(const float* w, int cin, int cout, int CIN, int mirror, void* out, hipStream_t s) {
    hipLaunchKernelGGL(k_swizzle_weights, dim3(28), dim3(256), 0, s, w, cin, cout, CIN, mirror,
                       static_cast<uint16_t*>(out));
    return hipGetLastError();
}

int conv_swizzle_elems(int CIN) { return (CIN == 16 ? 14 : 2) * 64 * 8; }

}  // namespace pcgmi
