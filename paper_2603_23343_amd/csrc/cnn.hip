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
// (k_conv3d_z): a work-group owns a 16 x 8 footprint and a chunk of planes,
// stages each input plane with its x/y halo in LDS once per chunk, and feeds
// each fragment it reads to the three output planes the input plane touches.
// The 2-channel input layer stages a
// 16 x 8 x 4 output block with its one-voxel halo (18 x 10 x 6 voxels) per
// work-group (k_conv3d). Each lane stores its voxel's 4 channels (8 bytes),
// so a tile's 16 voxels x 16 channels leave as 512 contiguous bytes.
//
// The transposed convolution of the backward pass (input gradient) is the
// same kernels with the taps mirrored and Cin/Cout swapped in the swizzle.
#include <hip/hip_runtime.h>

#include <algorithm>
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
    static_assert(CIN == 2, "the 16-channel input layers have their own chunking (ZP_NCH)");
    static constexpr int CHUNKS = 2;  // 32-wide K chunks: 16 taps x 2 channels (27 taps padded to 32)
};

// Output block per work-group and its input halo block.
constexpr int CB_X = 16, CB_Y = 8, CB_Z = 4;
constexpr int CH_X = CB_X + 2, CH_Y = CB_Y + 2, CH_Z = CB_Z + 2;
constexpr int CH_VOX = CH_X * CH_Y * CH_Z;
constexpr int CB_ROWS = CB_Y * CB_Z;                 // 16-voxel x-rows (tiles) per block
constexpr int CB_TILES = CB_ROWS / CONV_WAVES;       // tiles per wavefront

// Network input value of voxel i: (bf16(r[i] / rms), bf16(g[i])), rms =
// sqrt(rr / nvox) from a device scalar ||r||^2 (rr) or 1 when rr is null;
// g null reads as zero. Low half first.
template <typename T>
__device__ __forceinline__ uint32_t pack_voxel(const T* __restrict__ r, const float* __restrict__ g, float inv,
                                               int64_t i) {
    const float a = (float)to_c(r[i]) * inv;
    const float b = g ? g[i] : 0.f;
    return (uint32_t)f32_to_bf16_bits(a) | ((uint32_t)f32_to_bf16_bits(b) << 16);
}

// The 2-channel input layer: one 16 x 8 x 4 block of outputs per work-group.
// in: [nvox][CIN] bf16 bits. wsw: [CHUNKS][64 lanes][8] bf16 bits (the A operand).
// With TR non-void the layer packs its input itself: the halo is read from
// r (type TR) and g as pack_voxel forms it, and `in` is unused (inference:
// one pass over r and g instead of a packing pass and a pass over its output).
template <int CIN, int MODE, typename TR = void>
__global__ void __launch_bounds__(CONV_NT) k_conv3d(Dims d, int nbx, int nby, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                    const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                    double scale_mul, const TR* __restrict__ rsrc = nullptr,
                                                    const float* __restrict__ gsrc = nullptr,
                                                    const double* __restrict__ rr = nullptr) {
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
    float inv = 1.f;
    if constexpr (!std::is_void_v<TR>) inv = rr ? (float)(1.0 / sqrt(*rr / (double)d.nvox)) : 1.f;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int vox = halo_voxel(tid + j * CONV_NT, ok[j]);
        if constexpr (std::is_void_v<TR>) v[j] = *reinterpret_cast<const uint32_t*>(in + (size_t)vox * 2);
        else v[j] = pack_voxel(rsrc, gsrc, inv, vox);
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

// 16-channel input, marching up z with plane reuse. A work-group owns a
// 16 x 8 footprint of output voxels and a chunk of zc output planes, and
// walks the input planes p = z0 - 1 .. z1: each plane, with its one-voxel
// x/y halo (18 x 10 voxels), is staged in LDS once, and every patch fragment
// read from it feeds the three output planes that plane touches: p + 1 (tap
// dz = -1), p (dz = 0) and p - 1 (dz = +1), each with its own weights. A K
// chunk pairs two of a plane's 9 in-plane taps (padded to 10), so a plane
// costs a wavefront 10 fragment reads and 30 MFMAs, against 28 of each per
// output plane when each output plane gathers its 27 taps itself. Output
// plane p - 1 is complete after plane p and leaves from registers.
// One output channel (the last layer, OUT_SCALED_F32): the products are
// P W (patch rows as the A operand, weights as B) and the three output
// planes a fragment feeds are three columns of one accumulator: output
// plane o lives in column (o - z0 + 1) mod 3, the weights come in three
// column rotations, and after plane p the column of plane p - 1 is stored
// and cleared for plane p + 2. A plane then costs 10 MFMAs instead of 30.
// Pipeline: during plane p the load of plane p + 2 is in flight in one
// register set while the other (plane p + 1, loaded during plane p - 1) is
// stored into the LDS slot plane p - 1 used; one barrier per plane. The step
// has no branch around its loads and LDS stores (pieces outside the grid or
// past the chunk read a zero page, spare pieces write a dummy area), so the
// compiler waits only for the previous plane's loads before the LDS stores
// (with branches there it waited for every load in flight, the one just
// issued included). The slots' channel halves sit 3072 bytes apart (a
// multiple of 256): with halves 17280 bytes apart the fragment reads took
// 1.6x as long (bank conflicts, measured). Wavefront w computes the plane's
// x-rows w and w + 4. Same operand layout, epilogues and results as
// k_conv3d<16, MODE>; the weights come in 15 chunks: (dz index, in-plane
// pair) as the A operand, or for one output channel (column rotation,
// in-plane pair) as the B operand.
constexpr int ZC_OCC = 3;               // resident work-groups per CU (<= 168 VGPRs, 14.7 KB of LDS)
constexpr int ZS_HALF = 3072;           // one channel half of a plane slot: 18 x 10 x 16 bytes, padded to 256 B
constexpr int ZS_SLOT = 2 * ZS_HALF;    // a plane slot: both halves
constexpr int ZP_PAIRS = 5;             // in-plane tap pairs (9 taps + 1 zero-weight pad)
constexpr int ZP_NCH = 3 * ZP_PAIRS;    // weight chunks
constexpr int ZP_PIECES = CH_Y * CH_X * 2;              // 16-byte loads per plane (360)
constexpr int ZP_PPT = (ZP_PIECES + CONV_NT - 1) / CONV_NT;  // per thread (2)
constexpr int ZP_DUMMY = (ZP_PPT * CONV_NT - ZP_PIECES) * 16;  // LDS bytes for the spare pieces

template <int MODE>
__global__ void __launch_bounds__(CONV_NT, ZC_OCC) k_conv3d_z(Dims d, int nbx, int nby, int zc, const uint16_t* __restrict__ in,
                                                            const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                            const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                            double scale_mul, const void* __restrict__ zeros) {
    constexpr bool ONE = MODE == OUT_SCALED_F32;
    static_assert(CH_X * CH_Y * 16 <= ZS_HALF && ZS_HALF % 256 == 0, "plane slot layout");
    static_assert(CB_Y == 2 * CONV_WAVES && ZP_PPT == 2 && ZP_PIECES > CONV_NT, "piece mapping");
    __shared__ __attribute__((aligned(16))) unsigned char slots[2 * ZS_SLOT + ZP_DUMMY];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned nblk = gridDim.x;
    const unsigned lb = nblk % 8 == 0 ? (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8 : blockIdx.x;
    const int bx = (int)(lb % nbx), by = (int)((lb / nbx) % nby), bz = (int)(lb / (nbx * nby));
    const int x0 = bx * CB_X, y0 = by * CB_Y, z0 = bz * zc;
    const int z1 = min(z0 + zc, d.nz);

    bf16x8_t bw[ZP_NCH];
#pragma unroll
    for (int c = 0; c < ZP_NCH; ++c) bw[c] = *reinterpret_cast<const bf16x8_t*>(wsw + ((size_t)c * 64 + lane) * 8);

    // Plane staging: piece i = tid + 256 j (< 360) is channel half i % 2 of
    // halo voxel (i / 2) % 18 of halo row i / 36 (a row is 18 voxels x 32
    // bytes, contiguous in memory). Pieces outside the grid read the zero
    // page; pieces i >= 360 (j = 1, tid >= 104) read it too and land in the
    // dummy area. (16-byte units; voxel indices fit in 31 bits, which the
    // launcher checks. HIP's uint4 kept the register sets on the stack.)
    typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
    const u32x4_t* in4 = reinterpret_cast<const u32x4_t*>(in);
    const u32x4_t* zero4 = reinterpret_cast<const u32x4_t*>(zeros);
    const size_t plane4 = (size_t)d.nx * d.ny * 2;
    const int zend = min(z1 + 1, d.nz);  // planes [z0 - 1, zend) are read; the rest are zero
    unsigned pgoff[ZP_PPT];
    bool pxy[ZP_PPT];
    int pbase[ZP_PPT], pstride[ZP_PPT];
#pragma unroll
    for (int j = 0; j < ZP_PPT; ++j) {
        const int i = tid + CONV_NT * j, r = i / (2 * CH_X), hx = (i >> 1) % CH_X, hf = i & 1;
        const int gx = x0 + hx - 1, gy = y0 + r - 1;
        pxy[j] = (i < ZP_PIECES) & ((unsigned)gx < (unsigned)d.nx) & ((unsigned)gy < (unsigned)d.ny);
        pgoff[j] = pxy[j] ? (unsigned)(gy * d.nx + gx) * 2u + (unsigned)hf : 0u;
        const bool live = i < ZP_PIECES;
        pbase[j] = live ? hf * ZS_HALF + (r * CH_X + hx) * 16 : 2 * ZS_SLOT + (i - ZP_PIECES) * 16;
        pstride[j] = live ? ZS_SLOT : 0;
    }
    struct PlaneRegs {
        u32x4_t v[ZP_PPT];
    };
    auto fetch_plane = [&](int gz, PlaneRegs& pr) {
        const bool zok = gz >= 0 && gz < zend;
#pragma unroll
        for (int j = 0; j < ZP_PPT; ++j) {
            const u32x4_t* src = (pxy[j] & zok) ? in4 + ((size_t)gz * plane4 + pgoff[j]) : zero4;
            pr.v[j] = *src;
        }
    };
    auto store_plane = [&](int slot, const PlaneRegs& pr) {
#pragma unroll
        for (int j = 0; j < ZP_PPT; ++j)
            *reinterpret_cast<u32x4_t*>(slots + pbase[j] + slot * pstride[j]) = pr.v[j];
    };

    const int row = lane & 15, kgrp = lane >> 4;
    // the lane's channel half and x-row of the tiles: rows wu and wu + 4
    const int lane_off = (kgrp & 1) * ZS_HALF + (wu * CH_X + row) * 16;
    // in-plane tap s = 3 (dy + 1) + (dx + 1) of the lane in pair c: 2 c + (kgrp >> 1)
    int toff[ZP_PAIRS];
#pragma unroll
    for (int c = 0; c < ZP_PAIRS; ++c) {
        const int s = 2 * c + (kgrp >> 1);
        toff[c] = lane_off + (s < 9 ? ((s / 3) * CH_X + s % 3) * 16 : 0);  // the pad tap has zero weights
    }
    float scale = 0.f;
    if constexpr (ONE) scale = (float)(scale_rms2 ? sqrt(*scale_rms2) * scale_mul : scale_mul);
    // fragment reads of pair c from the slot at sb: tiles 0 and 1 (x-rows wu, wu + 4)
    auto frag = [&](const unsigned char* sb, int c, bf16x8_t (&a)[2]) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) a[tt] = *reinterpret_cast<const bf16x8_t*>(sb + toff[c] + tt * 4 * CH_X * 16);
    };

    // 16 output channels. Output plane o from its finished accumulators:
    // lane (kgrp, row) holds channels 4 kgrp .. + 3 of voxel `row` of tile tt
    // (x-row wu + 4 tt).
    auto emit16 = [&](int o, const f32x4_t (&acc)[2]) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int gy = y0 + wu + 4 * tt, gxo = x0 + row;
            if (gy >= d.ny || gxo >= d.nx) continue;
            const size_t v = (size_t)((o * d.ny + gy) * d.nx) + gxo;
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
    };
    // Input plane p: accumulate into nw (output p + 1, started here), md
    // (output p) and dn (output p - 1, finished here). Outputs outside
    // [z0, z1) are computed and dropped: their accumulators restart as nw.
    // Plane p + 1 goes into the slot plane p - 1 used (its last reads were at
    // plane p - 1, before that step's barrier); at p = z1 that store is dead.
    auto step16 = [&](int p, PlaneRegs& ld, const PlaneRegs& st, f32x4_t (&nw)[2], f32x4_t (&md)[2],
                      f32x4_t (&dn)[2]) {
        fetch_plane(p + 2, ld);
        nw[0] = nw[1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const unsigned char* sb = slots + (p & 1) * ZS_SLOT;
#pragma unroll
        for (int c = 0; c < ZP_PAIRS; ++c) {
            bf16x8_t a[2];
            frag(sb, c, a);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                nw[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], a[tt], nw[tt], 0, 0, 0);
                md[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[ZP_PAIRS + c], a[tt], md[tt], 0, 0, 0);
                dn[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[2 * ZP_PAIRS + c], a[tt], dn[tt], 0, 0, 0);
            }
        }
        store_plane((p + 1) & 1, st);
        if (p - 1 >= z0) emit16(p - 1, dn);
        __syncthreads();
    };
    // One output channel: D = P W, lane (kgrp, row) holds voxels 4 kgrp .. + 3
    // of the tile in column `row`. Step q = p - z0 + 1 uses the weight
    // rotation R = q mod 3: column (R + 1) mod 3 takes dz = -1 (output p + 1),
    // column R dz = 0 (output p), column (R + 2) mod 3 dz = +1 (output
    // p - 1, complete after this step: stored, then cleared).
    auto step1 = [&](int p, auto rot, PlaneRegs& ld, const PlaneRegs& st, f32x4_t (&acc)[2]) {
        constexpr int R = decltype(rot)::value;
        fetch_plane(p + 2, ld);
        const unsigned char* sb = slots + (p & 1) * ZS_SLOT;
#pragma unroll
        for (int c = 0; c < ZP_PAIRS; ++c) {
            bf16x8_t a[2];
            frag(sb, c, a);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt)
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[tt], bw[R * ZP_PAIRS + c], acc[tt], 0, 0, 0);
        }
        store_plane((p + 1) & 1, st);
        constexpr int done = (R + 2) % 3;
        const int o = p - 1;
        const bool vec = (d.nx & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
        if (o >= z0 && row == done) {
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int gy = y0 + wu + 4 * tt, gx = x0 + 4 * kgrp;
                if (gy >= d.ny) continue;
                float* dst = static_cast<float*>(out) + (size_t)((o * d.ny + gy) * d.nx) + gx;
                if (vec && gx + 3 < d.nx) {
                    *reinterpret_cast<float4*>(dst) =
                        make_float4(scale * acc[tt][0], scale * acc[tt][1], scale * acc[tt][2], scale * acc[tt][3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (gx + i < d.nx) dst[i] = scale * acc[tt][i];
                }
            }
        }
        if (row == done) acc[0] = acc[1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        __syncthreads();
    };

    // prologue: plane z0 - 1 into its slot, plane z0 into register set A
    PlaneRegs ra, rb;
    fetch_plane(z0 - 1, ra);
    store_plane((z0 - 1) & 1, ra);
    fetch_plane(z0, ra);
    __syncthreads();
    // Register sets rotate with period 2 (plane z0 - 1 + q loads into rb for
    // even q), accumulator sets (16 channels) or weight rotations (one
    // channel) with period 3: plane z0 - 1 + q uses nw = S[q % 3],
    // md = S[(q + 2) % 3], dn = S[(q + 1) % 3].
    if constexpr (ONE) {
        f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
        using R0 = std::integral_constant<int, 0>;
        using R1 = std::integral_constant<int, 1>;
        using R2 = std::integral_constant<int, 2>;
        for (int p = z0 - 1; p <= z1; p += 6) {
            step1(p, R0{}, rb, ra, acc);
            if (p + 1 > z1) break;
            step1(p + 1, R1{}, ra, rb, acc);
            if (p + 2 > z1) break;
            step1(p + 2, R2{}, rb, ra, acc);
            if (p + 3 > z1) break;
            step1(p + 3, R0{}, ra, rb, acc);
            if (p + 4 > z1) break;
            step1(p + 4, R1{}, rb, ra, acc);
            if (p + 5 > z1) break;
            step1(p + 5, R2{}, ra, rb, acc);
        }
    } else {
        f32x4_t S0[2], S1[2], S2[2];
        S1[0] = S1[1] = S2[0] = S2[1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        for (int p = z0 - 1; p <= z1; p += 6) {
            step16(p, rb, ra, S0, S2, S1);
            if (p + 1 > z1) break;
            step16(p + 1, ra, rb, S1, S0, S2);
            if (p + 2 > z1) break;
            step16(p + 2, rb, ra, S2, S1, S0);
            if (p + 3 > z1) break;
            step16(p + 3, ra, rb, S0, S2, S1);
            if (p + 4 > z1) break;
            step16(p + 4, rb, ra, S1, S0, S2);
            if (p + 5 > z1) break;
            step16(p + 5, ra, rb, S2, S1, S0);
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
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) out[i] = pack_voxel(r, g, inv, i);
}

// Swizzle FP32 master weights W[27][cin][cout] into the A-operand lane
// layout of the convolution for input width CIN (2: k_conv3d's chunks of 16
// taps; 16: k_conv3d_z's chunks of two in-plane taps of one dz, or with one
// output channel its B-operand column rotations; cin <= CIN, cout <= 16,
// missing entries zero). mirror: use W[26 - t][co][ci] (input gradient:
// mirrored taps, input and output channels swapped).
__global__ void k_swizzle_weights(const float* __restrict__ w, int cin, int cout, int CIN, int mirror,
                                  uint16_t* __restrict__ out) {
    const int nch = CIN == 16 ? ZP_NCH : ConvK<2>::CHUNKS;
    const int total = nch * 64 * 8;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int j = idx % 8, lane = (idx / 8) % 64, c = idx / 512;
        int n = lane & 15;
        const int k = 8 * (lane >> 4) + j;  // A[n][k] (or B[k][n] for one output channel)
        int tap, ci;
        if (CIN == 16 && !mirror && cout == 1) {
            // one output channel, the B operand: chunk 5 R + pr, column n of
            // rotation R holds dz = -1 (n = (R + 1) mod 3), 0 (n = R) or +1
            // (n = (R + 2) mod 3) of in-plane taps 2 pr, 2 pr + 1
            const int R = c / ZP_PAIRS, s = 2 * (c % ZP_PAIRS) + k / 16;
            const int dzi = n == (R + 1) % 3 ? 0 : n == R ? 1 : n == (R + 2) % 3 ? 2 : -1;
            tap = s < 9 && dzi >= 0 ? 9 * dzi + s : 27;
            ci = k % 16;
            n = 0;
        } else if (CIN == 16) {
            // chunk 5 dzi + pr: in-plane taps 2 pr, 2 pr + 1 of plane dz = dzi - 1
            const int s = 2 * (c % ZP_PAIRS) + k / 16;
            tap = s < 9 ? 9 * (c / ZP_PAIRS) + s : 27;
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

// Compute units of the current device (cached per device).
hipError_t conv_device_cus(int* ncu) {
    static int cache[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64 && cache[dev] > 0) {
        *ncu = cache[dev];
        return hipSuccess;
    }
    e = hipDeviceGetAttribute(ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && dev >= 0 && dev < 64) cache[dev] = *ncu;
    return e;
}

hipError_t launch_conv3d(int nx, int ny, int nz, int cin, int mode, const void* in, const void* wsw, void* out,
                         const void* mask, const double* scale_rms2, double scale_mul, const void* zeros, hipStream_t s) {
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
    hipLaunchKernelGGL((k_conv3d_z<MO>), dim3((unsigned)nbzm), dim3(CONV_NT), 0, s, d, nbx, nby, zc, in16, w16, out, \
                       m16, scale_rms2, scale_mul, zeros)
    if (cin == 16) {
        // z chunk: when the footprints alone are fewer than the resident
        // work-groups, split z so the grid fills them once (at 128^3: 128
        // footprints x 6 chunks of 22 planes = 768 = 3 per CU); chunks stay
        // within 8 .. 32 planes (each costs two extra input planes).
        int ncu = 0;
        if (conv_device_cus(&ncu) != hipSuccess) return hipErrorInvalidDevice;
        // (the one-channel kernel fits 128 VGPRs: four work-groups per CU)
        const int64_t fp = (int64_t)nbx * nby, slots = (int64_t)(mode == OUT_SCALED_F32 ? 4 : ZC_OCC) * ncu;
        const int64_t nzc = fp >= slots ? 1 : slots / fp;
        const int zc = (int)std::min<int64_t>(32, std::max<int64_t>(8, (nz + nzc - 1) / nzc));
        const int64_t nbzm = fp * ((nz + zc - 1) / zc);
        if (nbzm > INT32_MAX) return hipErrorInvalidValue;
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

// The first layer (2 -> 16, ReLU) straight from r (F32, F64 or BF16) and g.
hipError_t launch_conv3d_input(int nx, int ny, int nz, int dt, const void* r, const float* g, const double* rr,
                               const void* wsw, void* out, hipStream_t s) {
    Dims d{nx, ny, nz, (int64_t)nx * ny * nz};
    if (d.nvox == 0) return hipSuccess;
    const int nbx = (nx + CB_X - 1) / CB_X, nby = (ny + CB_Y - 1) / CB_Y, nbz = (nz + CB_Z - 1) / CB_Z;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    if (nb > INT32_MAX || d.nvox > INT32_MAX) return hipErrorInvalidValue;
    auto w16 = static_cast<const uint16_t*>(wsw);
#define PCGMI_CONVIN(T) \
    hipLaunchKernelGGL((k_conv3d<2, OUT_RELU_BF16, T>), dim3((unsigned)nb), dim3(CONV_NT), 0, s, d, nbx, nby, \
                       nullptr, w16, out, nullptr, nullptr, 1.0, static_cast<const T*>(r), g, rr)
    if (dt == DT_F32) PCGMI_CONVIN(float);
    else if (dt == DT_F64) PCGMI_CONVIN(double);
    else if (dt == DT_BF16) PCGMI_CONVIN(bf16);
    else return hipErrorInvalidValue;
#undef PCGMI_CONVIN
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

int conv_swizzle_elems(int CIN) { return (CIN == 16 ? ZP_NCH : ConvK<2>::CHUNKS) * 64 * 8; }

}  // namespace pcgmi
