// cnn.hip -- the learned preconditioner's network on gfx950: 3x3x3
// convolutions with zero padding as implicit GEMM on the matrix cores, plus
// the pieces of its training step.
//
// Layout. Activations are NDHWC: voxel-major [nz][ny][nx], channels
// innermost, BF16. A layer's FP32 master weight is W[27][Cin][Cout], tap
// t = 9 dz + 3 dy + dx (offsets -1..1). The network is 2 -> 16 -> 16 -> 16
// -> 1 with ReLU after the first three layers.
//
// Forward conv (implicit GEMM): voxels x Cout = 16, K = 27 * Cin, computed
// transposed: one v_mfma_f32_16x16x32_bf16 multiplies a 16 x 32 block of the
// weights (16 output channels x 32 values of K, the A operand) by a 32 x 16
// block of the patch matrix (32 values of K x 16 voxels, B). Operand lane
// layout (lane l): A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16] for
// j < 8, D[4 (l / 16) + i][l % 16] for i < 4: lane l reads K values of voxel
// l % 16 and ends with output channels 4 (l / 16) .. + 3 of that voxel. For
// Cin = 16 a K chunk covers two taps, so each lane's 8 patch values are 8
// consecutive channels of one neighbour: one 16-byte LDS load. For Cin = 2
// (the packed input) a chunk covers 16 taps and a lane gathers four (tap,
// 2-channel) pairs. Taps beyond 27 have zero weights; neighbours outside the
// grid are staged as zero. Weights are pre-swizzled into exactly the A lane
// layout, so each lane reads its 16 bytes per chunk with one load and keeps
// all chunks in registers. A work-group owns a 16 x 8 x 4 block of output
// voxels: it stages the block's input with its one-voxel halo (18 x 10 x 6
// voxels) in LDS once, so every input voxel crosses L2 about twice instead of
// 27 times, and each wavefront computes 8 tiles of 16 voxels (x-rows of the
// block) from LDS. Each lane stores its voxel's 4 channels (8 bytes), so a
// tile's 16 voxels x 16 channels leave as 512 contiguous bytes.
//
// The transposed convolution of the backward pass (input gradient) is the
// same kernel with the taps mirrored and Cin/Cout swapped in the swizzle.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pcgmi {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

constexpr int CONV_WAVES = 4;     // wavefronts per work-group
constexpr int CONV_NT = 64 * CONV_WAVES;

__device__ __forceinline__ uint16_t bf16_bits(float f) { return f32_to_bf16_bits(f); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// Two floats to BF16 (round to nearest even) in one conversion, low half first.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    typedef __attribute__((ext_vector_type(2))) float f2_t;
    typedef __attribute__((ext_vector_type(2))) __bf16 b2_t;
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{lo, hi}, b2_t));
}

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

// in: [nvox][CIN] bf16 bits. wsw: [CHUNKS][64 lanes][8] bf16 bits (the A operand).
template <int CIN, int MODE>
__global__ void __launch_bounds__(CONV_NT) k_conv3d(Dims d, int nbx, int nby, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                    const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                    double scale_mul) {
    constexpr int NCH = ConvK<CIN>::CHUNKS;
    constexpr int VB = CIN * 2;  // bytes per staged voxel (32 or 4)
    // CIN = 16: two planes of 16-byte channel halves, the second 17408 bytes
    // in (a multiple of 256): measured on MI355X, with the planes 17280 bytes
    // apart each of the products' ds_read_b128 took 1.6x as long (bank conflicts)
    constexpr int HPLANE = CH_VOX * 16 + 128;
    __shared__ __attribute__((aligned(16))) unsigned char halo[CIN == 16 ? 2 * HPLANE : CH_VOX * VB];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // XCD-aware order: work-group b runs on XCD b mod 8, so with a grid that
    // is a multiple of 8 each XCD takes a contiguous range of blocks, whose
    // shared halo voxels then meet in that XCD's L2.
    const unsigned nblk = gridDim.x;
    const unsigned lb = nblk % 8 == 0 ? (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8 : blockIdx.x;
    const int bx = (int)(lb % nbx), by = (int)((lb / nbx) % nby), bz = (int)(lb / (nbx * nby));
    const int x0 = bx * CB_X, y0 = by * CB_Y, z0 = bz * CB_Z;

    // A operands: all weight chunks in registers (loads issued first, so
    // they are in flight together with the halo loads).
    bf16x8_t bw[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) bw[c] = *reinterpret_cast<const bf16x8_t*>(wsw + ((size_t)c * 64 + lane) * 8);

    // Stage the halo block (zero outside the grid). Every load of a thread
    // is issued before its first LDS store, so a work-group waits for one
    // load latency, not one per piece (a loop that stored each piece before
    // loading the next serialised them).
    // Voxel offsets are 32-bit (the launcher checks the grid size); a piece
    // outside the grid or past the block loads voxel 0 and stores zero, so
    // every load is issued without a branch.
    auto halo_voxel = [&](int h, bool& ok) {
        const int hx = h % CH_X, hr = h / CH_X, hy = hr % CH_Y, hz = hr / CH_Y;
        const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
        // bitwise, not short-circuit: a select, not a branch per piece
        ok = (h < CH_VOX) & ((unsigned)gx < (unsigned)d.nx) & ((unsigned)gy < (unsigned)d.ny) &
             ((unsigned)gz < (unsigned)d.nz);
        const int vox = (gz * d.ny + gy) * d.nx + gx;
        return ok ? vox : 0;
    };
    if constexpr (CIN == 16) {
        // Wavefront w stages halo rows w, w + 4, ...: a row is 18 voxels x 32
        // bytes, contiguous in memory, loaded by lanes 0-35 (16 bytes each);
        // the row's coordinates are wave-uniform, so each load costs a few
        // vector instructions.
        constexpr int RPW = CH_Y * CH_Z / CONV_WAVES;
        static_assert(RPW * CONV_WAVES == CH_Y * CH_Z, "halo rows per wavefront");
        const int wu = __builtin_amdgcn_readfirstlane(wid);
        const int hx = lane >> 1, half = lane & 1, gx = x0 + hx - 1;
        const bool xok = lane < 2 * CH_X && (unsigned)gx < (unsigned)d.nx;
        // two batches of rows keep the staging registers below the compute's
        constexpr int B1 = (RPW + 1) / 2;
        auto stage_rows = [&](auto first, auto count) {
            constexpr int J0 = decltype(first)::value, NJ = decltype(count)::value;
            uint4 v[NJ];
            bool ok[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int r = wu + CONV_WAVES * (J0 + j), hy = r % CH_Y, hz = r / CH_Y;
                const int gy = y0 + hy - 1, gz = z0 + hz - 1;
                ok[j] = xok & ((unsigned)gy < (unsigned)d.ny) & ((unsigned)gz < (unsigned)d.nz);
                const int vox = ok[j] ? (gz * d.ny + gy) * d.nx + gx : 0;
                v[j] = *reinterpret_cast<const uint4*>(in + (size_t)vox * 16 + 8 * half);
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int r = wu + CONV_WAVES * (J0 + j);
                // channel halves in separate planes: a wavefront's 16 lanes of
                // one half read 16 consecutive 16-byte slots
                if (lane < 2 * CH_X)
                    *reinterpret_cast<uint4*>(halo + (size_t)half * HPLANE + (size_t)(r * CH_X + hx) * 16) =
                        ok[j] ? v[j] : make_uint4(0, 0, 0, 0);
            }
        };
        stage_rows(std::integral_constant<int, 0>{}, std::integral_constant<int, B1>{});
        stage_rows(std::integral_constant<int, B1>{}, std::integral_constant<int, RPW - B1>{});
    } else {
        constexpr int NP = (CH_VOX + CONV_NT - 1) / CONV_NT;
        uint32_t v[NP];
        bool ok[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int vox = halo_voxel(tid + j * CONV_NT, ok[j]);
            v[j] = *reinterpret_cast<const uint32_t*>(in + (size_t)vox * 2);
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int h = tid + j * CONV_NT;
            if (h < CH_VOX) *reinterpret_cast<uint32_t*>(halo + (size_t)h * 4) = ok[j] ? v[j] : 0u;
        }
    }

    __syncthreads();

    const int row = lane & 15, kgrp = lane >> 4;  // A: voxel row (x within the tile), K group of 8
    // Tile tt of wavefront wid is the block's x-row (yl, zl) = (wid + 4 (tt & 1),
    // tt / 2): the wavefront's part goes into a per-lane base address and the
    // tile's part is a constant, so every A-operand read is one LDS load at a
    // fixed offset from a few per-lane addresses. Taps past 26 read a voxel of
    // the block (any finite value): their weights are zero.
    static_assert(CB_Y == 2 * CONV_WAVES && CB_TILES == 2 * CB_Z, "tile mapping");
    auto tile_off = [](int tt) { return ((tt >> 1) * CH_Y + 4 * (tt & 1)) * CH_X; };
    auto tap_off = [](int t) { return t < 27 ? ((t / 9) * CH_Y + (t / 3) % 3) * CH_X + t % 3 : 0; };
    f32x4_t acc[CB_TILES];
#pragma unroll
    for (int tt = 0; tt < CB_TILES; ++tt) acc[tt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if constexpr (CIN == 16) {
        // lanes 0-31 take tap 2c, lanes 32-63 tap 2c + 1; channels 0-7 / 8-15 by (kgrp & 1)
        const unsigned char* hb = halo + (size_t)(kgrp & 1) * HPLANE + (size_t)(wid * CH_X + row) * 16;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const unsigned char* hc = hb + (size_t)((kgrp >> 1) ? tap_off(2 * c + 1) : tap_off(2 * c)) * 16;
#pragma unroll
            for (int tt = 0; tt < CB_TILES; ++tt) {
                const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(hc + (size_t)tile_off(tt) * 16);
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], a, acc[tt], 0, 0, 0);
            }
        }
    } else {
        // k = 2 tap + channel; the lane's 8 values: taps 16 c + 4 kgrp + (0..3), 2 channels each
        const unsigned char* hb = halo + (size_t)(wid * CH_X + row) * 4;
        int toff[NCH][4];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) toff[c][qq] = tap_off(16 * c + 4 * kgrp + qq);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
#pragma unroll
            for (int tt = 0; tt < CB_TILES; ++tt) {
                uint32_t w[4];
#pragma unroll
                for (int qq = 0; qq < 4; ++qq)
                    w[qq] = *reinterpret_cast<const uint32_t*>(hb + (size_t)(tile_off(tt) + toff[c][qq]) * 4);
                const bf16x8_t a = __builtin_bit_cast(bf16x8_t, make_uint4(w[0], w[1], w[2], w[3]));
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], a, acc[tt], 0, 0, 0);
            }
        }
    }

    // Results. The product is W^T P^T (weights as the A operand, the patch
    // rows as B, the same lane layouts), so lane (kgrp, row) holds output
    // channels 4 kgrp .. 4 kgrp + 3 of voxel `row` of the tile: each lane
    // writes its 4 channels as 8 bytes and a tile leaves as 512 contiguous
    // bytes, with no transpose through LDS.
    float scale = 0.f;
    if constexpr (MODE == OUT_SCALED_F32) scale = (float)(scale_rms2 ? sqrt(*scale_rms2) * scale_mul : scale_mul);
    const int wo = __builtin_amdgcn_readfirstlane(wid);
#pragma unroll
    for (int tt = 0; tt < CB_TILES; ++tt) {
        const int gy = y0 + wo + 4 * (tt & 1), gz = z0 + (tt >> 1), gx = x0 + row;
        if (!(gy < d.ny && gz < d.nz)) continue;  // wave-uniform
        if (gx >= d.nx) continue;
        const size_t v = (size_t)((gz * d.ny + gy) * d.nx) + gx;
        if constexpr (MODE == OUT_SCALED_F32) {
            if (kgrp == 0) static_cast<float*>(out)[v] = scale * acc[tt][0];
        } else {
            float val[4];
            uint2 m = make_uint2(0u, 0u);
            if constexpr (MODE == OUT_MASK_BF16) m = *reinterpret_cast<const uint2*>(mask + v * 16 + 4 * kgrp);
            const uint32_t mw[2] = {m.x, m.y};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                val[i] = acc[tt][i];
                if constexpr (MODE == OUT_RELU_BF16) val[i] = val[i] > 0.f ? val[i] : 0.f;
                if constexpr (MODE == OUT_MASK_BF16)
                    val[i] = bf16_val((uint16_t)((i & 1) ? mw[i >> 1] >> 16 : mw[i >> 1] & 0xffffu)) > 0.f ? val[i] : 0.f;
            }
            const uint2 o = make_uint2(pack_bf16x2(val[0], val[1]), pack_bf16x2(val[2], val[3]));
            *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + v * 16 + 4 * kgrp) = o;
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
    if (nb > INT32_MAX || d.nvox > INT32_MAX) return hipErrorInvalidValue;  // 32-bit voxel offsets
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
