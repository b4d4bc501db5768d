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
// all chunks in registers. The 16-channel input layers march up z
// (k_conv3d_z): a work-group owns a 16 x 8 footprint and a chunk of planes and
// keeps a ring of input planes with their x/y halo in LDS, so each input
// plane is staged once per chunk. The 2-channel input layer stages a
// 16 x 8 x 4 output block with its one-voxel halo (18 x 10 x 6 voxels) per
// work-group (k_conv3d). Each lane stores its voxel's 4 channels (8 bytes),
// so a tile's 16 voxels x 16 channels leave as 512 contiguous bytes.
//
// The transposed convolution of the backward pass (input gradient) is the
// same kernels with the taps mirrored and Cin/Cout swapped in the swizzle.
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

// The 2-channel input layer: one 16 x 8 x 4 block of outputs per work-group.
// in: [nvox][CIN] bf16 bits. wsw: [CHUNKS][64 lanes][8] bf16 bits (the A operand).
template <int CIN, int MODE>
__global__ void __launch_bounds__(CONV_NT) k_conv3d(Dims d, int nbx, int nby, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                    const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                    double scale_mul) {
    static_assert(CIN == 2, "the 16-channel input layers run k_conv3d_z");
    constexpr int NCH = ConvK<CIN>::CHUNKS;
    __shared__ __attribute__((aligned(16))) unsigned char halo[CH_VOX * 4];
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

// 16-channel input, marching up z. A work-group owns a 16 x 8 footprint of
// output voxels and a chunk of ZC_CONV output planes; it keeps the input
// planes z - 1, z, z + 1 (with their one-voxel x/y halo, 18 x 10 voxels) in a
// ring of four LDS plane slots, so each input plane is staged once per chunk
// instead of once per 4-plane block (a block per work-group, as the 2-channel
// kernel above, read 2.5x its input through the fabric: 18 x 10 x 6 halo
// voxels per 16 x 8 x 4 outputs; 44 -> 34 us per 16 -> 16 layer at 128^3).
// The slots' channel halves sit 3072 bytes apart (a multiple of 256): with
// halves 17280 bytes apart the products' ds_read_b128 took 1.6x as long
// (bank conflicts, measured).
// Step z computes output plane z from the three resident slots while plane
// z + 3 is loaded into one register set; the other set (plane z + 2, loaded
// during step z - 1) goes into the slot plane z - 2 used, then one barrier.
// (With one plane of look-ahead each step waited for its plane's load: the
// step's products are shorter than a load's latency.) Wavefront w computes
// the plane's x-rows w and w + 4.
// Same operand layout, epilogues and results as k_conv3d<16, MODE>.
constexpr int ZC_CONV = 16;
constexpr int ZS_HALF = 3072;           // one channel half of a plane slot: 18 x 10 x 16 bytes, padded to 256 B
constexpr int ZS_SLOT = 2 * ZS_HALF;    // a plane slot: both halves

template <int MODE>
__global__ void __launch_bounds__(CONV_NT, 4) k_conv3d_z(Dims d, int nbx, int nby, const uint16_t* __restrict__ in,
                                                      const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                      const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                      double scale_mul) {
    constexpr int NCH = ConvK<16>::CHUNKS;
    static_assert(CH_X * CH_Y * 16 <= ZS_HALF && ZS_HALF % 256 == 0, "plane slot layout");
    __shared__ __attribute__((aligned(16))) unsigned char slots[4 * ZS_SLOT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned nblk = gridDim.x;
    const unsigned lb = nblk % 8 == 0 ? (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8 : blockIdx.x;
    const int bx = (int)(lb % nbx), by = (int)((lb / nbx) % nby), bz = (int)(lb / (nbx * nby));
    const int x0 = bx * CB_X, y0 = by * CB_Y, z0 = bz * ZC_CONV;
    const int z1 = min(z0 + ZC_CONV, d.nz);

    bf16x8_t bw[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) bw[c] = *reinterpret_cast<const bf16x8_t*>(wsw + ((size_t)c * 64 + lane) * 8);

    // Plane staging: wavefront w takes halo rows w, w + 4, w + 8 (< 10) of a
    // plane; lanes 0-35 load one 16-byte channel half each (the row is 18
    // voxels x 32 bytes, contiguous). Points outside the grid load voxel 0
    // and are stored as zero.
    const int hx = lane >> 1, half = lane & 1, gx = x0 + hx - 1;
    const bool xok = lane < 2 * CH_X && (unsigned)gx < (unsigned)d.nx;
    constexpr int RPW = (CH_Y + CONV_WAVES - 1) / CONV_WAVES;  // 3
    struct PlaneRegs {
        uint4 v[RPW];
        bool ok[RPW];
    };
    auto fetch_plane = [&](int gz, PlaneRegs& pr) {
#pragma unroll
        for (int j = 0; j < RPW; ++j) {
            const int r = wu + CONV_WAVES * j, gy = y0 + r - 1;
            pr.ok[j] = xok & (r < CH_Y) & ((unsigned)gy < (unsigned)d.ny) & ((unsigned)gz < (unsigned)d.nz);
            const int vox = pr.ok[j] ? (gz * d.ny + gy) * d.nx + gx : 0;
            pr.v[j] = *reinterpret_cast<const uint4*>(in + (size_t)vox * 16 + 8 * half);
        }
    };
    auto store_plane = [&](int slot, const PlaneRegs& pr) {
        unsigned char* base = slots + (size_t)slot * ZS_SLOT + (size_t)half * ZS_HALF;
#pragma unroll
        for (int j = 0; j < RPW; ++j) {
            const int r = wu + CONV_WAVES * j;
            if (lane < 2 * CH_X && r < CH_Y)
                *reinterpret_cast<uint4*>(base + (size_t)(r * CH_X + hx) * 16) =
                    pr.ok[j] ? pr.v[j] : make_uint4(0, 0, 0, 0);
        }
    };
    // prologue: planes z0 - 1, z0, z0 + 1 into slots (plane + 4) % 4, plane
    // z0 + 2 into register set A
    PlaneRegs ra, rb;
    fetch_plane(z0 - 1, ra);
    fetch_plane(z0, rb);
    store_plane((z0 + 3) & 3, ra);
    store_plane(z0 & 3, rb);
    fetch_plane(z0 + 1, ra);
    store_plane((z0 + 1) & 3, ra);
    fetch_plane(z0 + 2, ra);
    __syncthreads();

    const int row = lane & 15, kgrp = lane >> 4;
    // the lane's channel half and x-row of the tiles: rows wu and wu + 4
    const int lane_off = (kgrp & 1) * ZS_HALF + (wu * CH_X + row) * 16;
    // per chunk, the lane's tap (2c or 2c + 1): its plane (dz) and in-plane offset
    auto tap_dz = [](int t) { return t < 27 ? t / 9 : 1; };
    auto tap_in = [](int t) { return t < 27 ? (((t / 3) % 3) * CH_X + t % 3) * 16 : 0; };
    float scale = 0.f;
    if constexpr (MODE == OUT_SCALED_F32) scale = (float)(scale_rms2 ? sqrt(*scale_rms2) * scale_mul : scale_mul);
    // step z: load plane z + 3 into `ld` (in flight during the products),
    // store plane z + 2 from `st`
    auto step = [&](int z, PlaneRegs& ld, const PlaneRegs& st) {
        if (z + 3 <= z1) fetch_plane(z + 3, ld);
        // slot offsets of planes z - 1, z, z + 1
        const int so[3] = {((z + 3) & 3) * ZS_SLOT, (z & 3) * ZS_SLOT, ((z + 1) & 3) * ZS_SLOT};
        f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int ta = 2 * c, tb = 2 * c + 1;
            const int off = (kgrp >> 1) ? so[tap_dz(tb)] + tap_in(tb) : so[tap_dz(ta)] + tap_in(ta);
            const unsigned char* pa = slots + lane_off + off;
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(pa + tt * 4 * CH_X * 16);
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], a, acc[tt], 0, 0, 0);
            }
        }
        // results of plane z: lane (kgrp, row) holds channels 4 kgrp .. + 3 of voxel `row`
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int gy = y0 + wu + 4 * tt, gxo = x0 + row;
            if (gy >= d.ny || gxo >= d.nx) continue;
            const size_t v = (size_t)((z * d.ny + gy) * d.nx) + gxo;
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
                *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + v * 16 + 4 * kgrp) =
                    make_uint2(pack_bf16x2(val[0], val[1]), pack_bf16x2(val[2], val[3]));
            }
        }
        // plane z + 2 goes into the slot plane z - 2 used (read by no one at
        // step z: the last reads of it were at step z - 1, before its barrier)
        if (z + 2 <= z1) store_plane((z + 2) & 3, st);
        __syncthreads();
    };
    for (int z = z0; z < z1; z += 2) {
        step(z, rb, ra);
        if (z + 1 < z1) step(z + 1, ra, rb);
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
#define PCGMI_CONVZ(MO) \
    hipLaunchKernelGGL((k_conv3d_z<MO>), dim3((unsigned)nbzm), dim3(CONV_NT), 0, s, d, nbx, nby, in16, w16, out, m16, \
                       scale_rms2, scale_mul)
    if (cin == 16) {
        const int64_t nbzm = (int64_t)nbx * nby * ((nz + ZC_CONV - 1) / ZC_CONV);
        switch (mode) {
            case OUT_RELU_BF16: PCGMI_CONVZ(OUT_RELU_BF16); break;
            case OUT_SCALED_F32: PCGMI_CONVZ(OUT_SCALED_F32); break;
            case OUT_MASK_BF16: PCGMI_CONVZ(OUT_MASK_BF16); break;
            case OUT_LINEAR_BF16: PCGMI_CONVZ(OUT_LINEAR_BF16); break;
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
#undef PCGMI_CONVZ
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
