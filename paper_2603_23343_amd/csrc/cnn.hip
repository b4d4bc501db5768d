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
// reads its 16 bytes per chunk with one load. A wavefront computes 4 tiles
// (64 consecutive voxels) and keeps all weight chunks in registers; the
// 16 x 16 FP32 results go through LDS so each voxel's 16 channels leave as
// two 16-byte stores.
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
constexpr int CONV_TILES = 4;     // 16-voxel tiles per wavefront
constexpr int CONV_NT = 64 * CONV_WAVES;

__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }
__device__ __forceinline__ uint16_t bf16_bits(float f) { return f32_to_bf16_bits(f); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

struct Dims {
    int nx, ny, nz;
    int64_t nvox;
};

// Linear index of the neighbour of voxel v at tap t, or -1 outside the grid.
__device__ __forceinline__ int64_t nb_index(const Dims& d, int x, int y, int z, int t) {
    const int xx = x + (t % 3) - 1, yy = y + (t / 3) % 3 - 1, zz = z + t / 9 - 1;
    if (xx < 0 || xx >= d.nx || yy < 0 || yy >= d.ny || zz < 0 || zz >= d.nz) return -1;
    return ((int64_t)zz * d.ny + yy) * d.nx + xx;
}

// Output modes of the conv kernel.
enum ConvOut : int {
    OUT_RELU_BF16 = 0,   // hidden layer: bf16(relu(D)), 16 channels
    OUT_SCALED_F32 = 1,  // last layer: out[v] = scale * D[v][0] (FP32, one channel)
    OUT_MASK_BF16 = 2,   // input gradient: bf16(D * (mask[v][c] > 0)), 16 channels
    OUT_LINEAR_BF16 = 3  // bf16(D), 16 channels
};

template <int CIN> struct ConvK {
    static constexpr int CHUNKS = CIN == 16 ? 14 : 2;  // 32-wide K chunks (27 taps padded)
};

// in: [nvox][CIN] bf16 bits. wsw: [CHUNKS][64 lanes][8] bf16 bits (B operand).
template <int CIN, int MODE>
__global__ void __launch_bounds__(CONV_NT) k_conv3d(Dims d, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                    const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                    double scale_mul) {
    constexpr int NCH = ConvK<CIN>::CHUNKS;
    __shared__ float lds_d[CONV_WAVES][16][17];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave_gid = (int64_t)blockIdx.x * CONV_WAVES + wid;
    const int64_t vbase = wave_gid * (16 * CONV_TILES);
    if (vbase >= d.nvox) return;  // whole wavefront past the end (no barrier below is block-wide)

    // B operands: all weight chunks in registers.
    bf16x8_t bw[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const uint16_t* p = wsw + ((size_t)c * 64 + lane) * 8;
        Vec16<bf16> raw = *reinterpret_cast<const Vec16<bf16>*>(p);
#pragma unroll
        for (int j = 0; j < 8; ++j) bw[c][j] = bits_to_bf16(raw.e[j].bits);
    }
    const int row = lane & 15, kgrp = lane >> 4;  // A: voxel row, K group of 8
    f32x4_t acc[CONV_TILES];
#pragma unroll
    for (int tt = 0; tt < CONV_TILES; ++tt) {
        acc[tt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const int64_t v = vbase + tt * 16 + row;
        const bool vok = v < d.nvox;
        const int64_t vv = vok ? v : 0;
        const int x = (int)(vv % d.nx), y = (int)((vv / d.nx) % d.ny), z = (int)(vv / ((int64_t)d.nx * d.ny));
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            bf16x8_t a;
            if constexpr (CIN == 16) {
                const int tap = 2 * c + (kgrp >> 1);
                const int ci0 = 8 * (kgrp & 1);
                const int64_t nb = (vok && tap < 27) ? nb_index(d, x, y, z, tap) : -1;
                Vec16<bf16> raw = *reinterpret_cast<const Vec16<bf16>*>(in + (nb >= 0 ? nb : 0) * 16 + ci0);
#pragma unroll
                for (int j = 0; j < 8; ++j) a[j] = bits_to_bf16(nb >= 0 ? raw.e[j].bits : (uint16_t)0);
            } else {
                // k = 2 tap + channel; lane's 8 values: taps 16 c + 4 kgrp + (0..3), 2 channels each
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int tap = 16 * c + 4 * kgrp + q;
                    const int64_t nb = (vok && tap < 27) ? nb_index(d, x, y, z, tap) : -1;
                    const uint32_t w2 = *reinterpret_cast<const uint32_t*>(in + (nb >= 0 ? nb : 0) * 2);
                    const uint32_t w = nb >= 0 ? w2 : 0u;
                    a[2 * q] = bits_to_bf16((uint16_t)(w & 0xffffu));
                    a[2 * q + 1] = bits_to_bf16((uint16_t)(w >> 16));
                }
            }
            acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[c], acc[tt], 0, 0, 0);
        }
    }
    // Results: lane holds D[4 kgrp + i][row] (voxel 4 kgrp + i, channel row).
    float scale = 0.f;
    if constexpr (MODE == OUT_SCALED_F32) scale = (float)(scale_rms2 ? sqrt(*scale_rms2) * scale_mul : scale_mul);
#pragma unroll
    for (int tt = 0; tt < CONV_TILES; ++tt) {
        const int64_t v0 = vbase + tt * 16;
        if constexpr (MODE == OUT_SCALED_F32) {
            if (row == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t v = v0 + 4 * kgrp + i;
                    if (v < d.nvox) static_cast<float*>(out)[v] = scale * acc[tt][i];
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
                const int64_t v = v0 + vi;
                if (v < d.nvox) {
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
    const int64_t waves = (d.nvox + 16 * CONV_TILES - 1) / (16 * CONV_TILES);
    const unsigned nb = (unsigned)((waves + CONV_WAVES - 1) / CONV_WAVES);
    if (nb == 0) return hipSuccess;
    auto in16 = static_cast<const uint16_t*>(in);
    auto w16 = static_cast<const uint16_t*>(wsw);
    auto m16 = static_cast<const uint16_t*>(mask);
#define PCGMI_CONV(CI, MO) \
    hipLaunchKernelGGL((k_conv3d<CI, MO>), dim3(nb), dim3(CONV_NT), 0, s, d, in16, w16, out, m16, scale_rms2, scale_mul)
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
