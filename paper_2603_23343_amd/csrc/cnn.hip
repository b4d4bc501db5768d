// cnn.hip -- the learned preconditioner's network on gfx950: 3x3x3
// convolutions with zero padding as implicit GEMM on the matrix cores, plus
// the pieces of its training step.
//
// Layout. Activations are NDHWC: voxel-major [nz][ny][nx], channels
// innermost, BF16. A layer's FP32 master weight is W[27][Cin][Cout], tap
// t = 9 dz + 3 dy + dx (offsets -1..1). The network is 2 -> 16 -> 16 -> 16
// -> 1 with ReLU after the first three layers.
//
// Convolution (implicit GEMM): voxels x Cout = 16, K = 27 * Cin, computed
// transposed: one v_mfma_f32_16x16x32_bf16 multiplies a 16 x 32 block of the
// weights (16 output channels x 32 values of K, the A operand) by a 32 x 16
// block of the patch matrix (32 values of K x 16 voxels, B). Operand lane
// layout (lane l): A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16] for
// j < 8, D[4 (l / 16) + i][l % 16] for i < 4: lane l reads K values of voxel
// l % 16 and ends with output channels 4 (l / 16) .. + 3 of that voxel. Every
// layer marches up z (k_conv3d_z): a work-group owns a 16 x 8 footprint and a
// chunk of planes, stages each input plane with its x/y halo in LDS once per
// chunk, and feeds each fragment it reads to the three output planes the
// input plane touches (taps dz = -1, 0, +1, each with its own weights). For
// Cin = 16 a K chunk covers two in-plane taps, so each lane's 8 patch values
// are 8 consecutive channels of one neighbour: one 16-byte LDS load. For
// Cin = 2 (the packed input) one chunk covers a plane's 9 in-plane taps and
// a lane gathers four (tap, 2-channel) words. Taps past the last have zero
// weights; neighbours outside the grid are staged as zero. Weights are
// pre-swizzled into exactly the operand lane layout, so each lane reads its
// 16 bytes per chunk with one load and keeps all chunks in registers. Each
// lane stores its voxel's 4 channels (8 bytes), so a tile's 16 voxels x 16
// channels leave as 512 contiguous bytes.
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

constexpr int CB_X = 16;                // footprint width: one 16-voxel tile row
constexpr int CH_X = CB_X + 2;          // halo row width

// Two floats to the network input's BF16 pair (low half first).
__device__ __forceinline__ uint32_t pack_pair(float a, float b) {
    return (uint32_t)f32_to_bf16_bits(a) | ((uint32_t)f32_to_bf16_bits(b) << 16);
}
// Network input value of voxel i: (bf16(r[i] / rms), bf16(g[i])), rms =
// sqrt(rr / nvox) from a device scalar ||r||^2 (rr) or 1 when rr is null;
// g null reads as zero.
template <typename T>
__device__ __forceinline__ uint32_t pack_voxel(const T* __restrict__ r, const float* __restrict__ g, float inv,
                                               int64_t i) {
    return pack_pair((float)to_c(r[i]) * inv, g ? g[i] : 0.f);
}

// Every layer marches up z with plane reuse. A work-group (ZW = 4
// wavefronts) owns a 16 x 8 footprint of output voxels and a chunk of zc
// output planes, and walks the input planes p = z0 - 1 .. z1: each plane,
// with its one-voxel x/y halo (18 x 10 voxels), is staged in LDS once, and
// every patch fragment read from it feeds the three output planes that plane
// touches: p + 1 (tap dz = -1), p (dz = 0) and p - 1 (dz = +1), each with its
// own weights. Output plane p - 1 is complete after plane p and leaves from
// registers.
//  * Cin = 16: a K chunk pairs two of a plane's 9 in-plane taps (padded to
//    10), so a plane costs a wavefront 10 fragment reads and 30 MFMAs,
//    against 28 of each per output plane when each output plane gathers its
//    27 taps itself. The slots' channel halves sit 3072 bytes apart (a
//    multiple of 256): with halves 17280 bytes apart the fragment reads took
//    1.6x as long (bank conflicts, measured).
//  * Cin = 2: one chunk holds the 9 in-plane taps x 2 channels (18 of 32 K
//    values), a lane gathers its four (tap, channel pair) words; 3 MFMAs
//    per tile and plane. With TR non-void the layer forms its input itself
//    from r (type TR) and g as pack_voxel does (inference: no packing pass).
//  * One output channel (the last layer, OUT_SCALED_F32, Cin = 16): the
//    products are P W (patch rows as the A operand, weights as B) and the
//    three output planes a fragment feeds are three columns of one
//    accumulator: output plane o lives in column (o - z0 + 1) mod 3, the
//    weights come in three column rotations, and after plane p the column of
//    plane p - 1 is stored and cleared for plane p + 2. A plane then costs 10
//    MFMAs instead of 30.
// Pipeline: during plane p the load of plane p + 2 is in flight in one
// register set while the other (plane p + 1, loaded during plane p - 1) is
// stored into the LDS slot plane p - 1 used; one barrier per plane. The step
// has no branch around its loads, LDS stores or (16-channel output) global
// stores: pieces outside the grid or past the chunk read a zero page, spare
// pieces write a dummy LDS area, outputs outside the grid go to a sink. With
// branches there the compiler could not count the memory operations in
// flight and waited for all of them, the plane load just issued included.
// Wavefront w computes the plane's x-rows w and w + 4.
constexpr int ZC_OCC = 3;               // wavefronts per SIMD (<= 168 VGPRs)
constexpr int ZW = 4;                   // wavefronts per work-group (one-wavefront groups without
                                        // barriers measured no faster)
constexpr int ZNT = 64 * ZW;
constexpr int ZROWS = 2 * ZW;           // output rows of a footprint (16 x 8)
constexpr int ZHROWS = ZROWS + 2;       // halo rows
constexpr int ZP_PAIRS = 5;             // in-plane tap pairs (9 taps + 1 zero-weight pad)
constexpr int CONV_SINK = 64 * 128 * 8; // bytes of the sink that takes stores outside the grid

// Plane staging per input width.
template <int CIN> struct ZPlane;
template <> struct ZPlane<16> {                                   // two 16-byte channel halves per voxel
    static constexpr int PIECE = 16;
    static constexpr int HALF = (ZHROWS * CH_X * 16 + 255) / 256 * 256;  // a channel half, padded to 256 B
    static constexpr int SLOT = 2 * HALF;
    static constexpr int PIECES = ZHROWS * CH_X * 2;              // 360
    static constexpr int NCH = 3 * ZP_PAIRS;                      // weight chunks: (dz, pair) or (rotation, pair)
};
template <> struct ZPlane<2> {                                    // one 4-byte word per voxel
    static constexpr int PIECE = 4;
    static constexpr int HALF = 0;
    static constexpr int SLOT = (ZHROWS * CH_X * 4 + 255) / 256 * 256;
    static constexpr int PIECES = ZHROWS * CH_X;                  // 180
    static constexpr int NCH = 3;                                 // weight chunks: dz
};
template <int CIN> constexpr int zppt() { return (ZPlane<CIN>::PIECES + ZNT - 1) / ZNT; }
template <int CIN> constexpr int zlds() {
    return 2 * ZPlane<CIN>::SLOT + (zppt<CIN>() * ZNT - ZPlane<CIN>::PIECES) * ZPlane<CIN>::PIECE;
}

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));  // (HIP's uint4 kept register sets on the stack)
// A plane in flight: the thread's 16-byte pieces (Cin = 16), its packed
// word (Cin = 2), or its raw r and g values (Cin = 2 formed in the layer).
template <int CIN, typename TR> struct ZRegs {
    u32x4_t v[zppt<16>()];
};
template <> struct ZRegs<2, void> {
    uint32_t v;
};
template <typename TR> struct ZRaw {
    TR r;
    float g;
    bool ok;
};
template <> struct ZRegs<2, float> : ZRaw<float> {};
template <> struct ZRegs<2, double> : ZRaw<double> {};
template <> struct ZRegs<2, bf16> : ZRaw<bf16> {};

template <int MODE, int CIN, typename TR>
__global__ void __launch_bounds__(ZNT, ZC_OCC) k_conv3d_z(Dims d, int nbx, int nby, int zc, const uint16_t* __restrict__ in,
                                                         const uint16_t* __restrict__ wsw, void* __restrict__ out,
                                                         const uint16_t* __restrict__ mask, const double* scale_rms2,
                                                         double scale_mul, const void* __restrict__ zeros,
                                                         void* __restrict__ sink, const TR* __restrict__ rsrc,
                                                         const float* __restrict__ gsrc, const double* rr_in) {
    constexpr bool ONE = MODE == OUT_SCALED_F32;
    constexpr bool RAW = !std::is_void_v<TR>;
    static_assert(CIN == 16 || CIN == 2, "input width");
    static_assert(!ONE || CIN == 16, "one output channel follows a 16-channel layer");
    static_assert(!RAW || CIN == 2, "only the first layer forms its input");
    using PL = ZPlane<CIN>;
    constexpr int PPT = zppt<CIN>();
    using PlaneRegs = ZRegs<CIN, TR>;
    __shared__ __attribute__((aligned(16))) unsigned char slots[zlds<CIN>()];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    // XCD-aware order: work-group b runs on XCD b mod 8, so with a grid that
    // is a multiple of 8 each XCD takes a contiguous range of footprints,
    // whose shared halo rows then meet in that XCD's L2.
    const unsigned nblk = gridDim.x;
    const unsigned lb = nblk % 8 == 0 ? (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8 : blockIdx.x;
    const int bx = (int)(lb % nbx), by = (int)((lb / nbx) % nby), bz = (int)(lb / (nbx * nby));
    const int x0 = bx * CB_X, y0 = by * ZROWS, z0 = bz * zc;
    const int z1 = min(z0 + zc, d.nz);

    bf16x8_t bw[PL::NCH];
#pragma unroll
    for (int c = 0; c < PL::NCH; ++c) bw[c] = *reinterpret_cast<const bf16x8_t*>(wsw + ((size_t)c * 64 + lane) * 8);

    // Plane staging. Cin = 16: piece i = tid + 256 j (< 360) is channel half
    // i % 2 of halo voxel (i / 2) % 18 of halo row i / 36 (a row is 18 voxels
    // x 32 bytes, contiguous in memory). Cin = 2: piece i = tid (< 180) is
    // halo voxel i % 18 of halo row i / 18. Pieces outside the grid read the
    // zero page (and, formed in the layer, are staged as zero); spare pieces
    // read it too and land in the dummy area. Offsets are in piece units;
    // voxel indices fit in 31 bits, which the launcher checks.
    const int zend = min(z1 + 1, d.nz);  // planes [z0 - 1, zend) are read; the rest are zero
    const size_t plane_pieces = (size_t)d.nx * d.ny * (CIN == 16 ? 2 : 1);
    unsigned pgoff[PPT];
    bool pxy[PPT];
    int pbase[PPT], pstride[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int i = tid + ZNT * j;
        const bool live = i < PL::PIECES;
        int r, hx, hf;
        if constexpr (CIN == 16) {
            r = i / (2 * CH_X), hx = (i >> 1) % CH_X, hf = i & 1;
        } else {
            r = i / CH_X, hx = i % CH_X, hf = 0;
        }
        const int gx = x0 + hx - 1, gy = y0 + r - 1;
        pxy[j] = live & ((unsigned)gx < (unsigned)d.nx) & ((unsigned)gy < (unsigned)d.ny);
        pgoff[j] = pxy[j] ? (unsigned)(gy * d.nx + gx) * (CIN == 16 ? 2u : 1u) + (unsigned)hf : 0u;
        pbase[j] = live ? hf * PL::HALF + (r * CH_X + hx) * PL::PIECE : 2 * PL::SLOT + (i - PL::PIECES) * PL::PIECE;
        pstride[j] = live ? PL::SLOT : 0;
    }
    float inv = 1.f;
    if constexpr (RAW) inv = rr_in ? (float)(1.0 / sqrt(*rr_in / (double)d.nvox)) : 1.f;
    const float* gsel = gsrc ? gsrc : static_cast<const float*>(zeros);
    auto fetch_plane = [&](int gz, PlaneRegs& pr) {
        const bool zok = gz >= 0 && gz < zend;
        if constexpr (CIN == 16) {
            const u32x4_t* in4 = reinterpret_cast<const u32x4_t*>(in);
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const u32x4_t* src = (pxy[j] & zok) ? in4 + ((size_t)gz * plane_pieces + pgoff[j])
                                                    : static_cast<const u32x4_t*>(zeros);
                pr.v[j] = *src;
            }
        } else if constexpr (!RAW) {
            const bool ok = pxy[0] & zok;
            pr.v = *(ok ? reinterpret_cast<const uint32_t*>(in) + ((size_t)gz * plane_pieces + pgoff[0])
                        : static_cast<const uint32_t*>(zeros));
        } else {
            pr.ok = pxy[0] & zok;
            const size_t vi = (size_t)gz * plane_pieces + pgoff[0];
            pr.r = *(pr.ok ? rsrc + vi : static_cast<const TR*>(zeros));
            pr.g = *((pr.ok && gsrc) ? gsel + vi : static_cast<const float*>(zeros));
        }
    };
    auto store_plane = [&](int slot, const PlaneRegs& pr) {
        if constexpr (CIN == 16) {
#pragma unroll
            for (int j = 0; j < PPT; ++j)
                *reinterpret_cast<u32x4_t*>(slots + pbase[j] + slot * pstride[j]) = pr.v[j];
        } else if constexpr (!RAW) {
            *reinterpret_cast<uint32_t*>(slots + pbase[0] + slot * pstride[0]) = pr.v;
        } else {
            const uint32_t w = pr.ok ? pack_pair((float)to_c(pr.r) * inv, pr.g) : 0u;
            *reinterpret_cast<uint32_t*>(slots + pbase[0] + slot * pstride[0]) = w;
        }
    };

    const int row = lane & 15, kgrp = lane >> 4;
    // Fragment offsets. Cin = 16: the lane's channel half and x-row, and per
    // pair c its in-plane tap s = 2 c + (kgrp >> 1), s = 3 (dy + 1) + (dx + 1).
    // Cin = 2: the lane's taps s = 4 kgrp + u, u < 4 (K values 8 kgrp .. + 7 =
    // (tap, channel) pairs). The pad taps have zero weights and read any
    // staged word.
    constexpr int NOFF = CIN == 16 ? ZP_PAIRS : 4;
    int toff[NOFF];
    {
        const int lane_off = (kgrp & 1) * PL::HALF + (wu * CH_X + row) * PL::PIECE;
#pragma unroll
        for (int c = 0; c < NOFF; ++c) {
            const int s = CIN == 16 ? 2 * c + (kgrp >> 1) : 4 * kgrp + c;
            toff[c] = (CIN == 16 ? lane_off : (wu * CH_X + row) * PL::PIECE) +
                      (s < 9 ? ((s / 3) * CH_X + s % 3) * PL::PIECE : 0);
        }
    }
    constexpr int TILE_STEP = ZW * CH_X * PL::PIECE;  // LDS distance of the wavefront's second x-row
    float scale = 0.f;
    if constexpr (ONE) scale = (float)(scale_rms2 ? sqrt(*scale_rms2) * scale_mul : scale_mul);
    // Cin = 16: the patch fragments of pair c for tiles 0 and 1.
    auto frag16 = [&](const unsigned char* sb, int c, bf16x8_t (&a)[2]) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) a[tt] = *reinterpret_cast<const bf16x8_t*>(sb + toff[c] + tt * TILE_STEP);
    };
    // Cin = 2: the lane's four words for tiles 0 and 1.
    auto frag2 = [&](const unsigned char* sb, bf16x8_t (&a)[2]) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            u32x4_t w;
#pragma unroll
            for (int u = 0; u < 4; ++u) w[u] = *reinterpret_cast<const uint32_t*>(sb + toff[u] + tt * TILE_STEP);
            a[tt] = __builtin_bit_cast(bf16x8_t, w);
        }
    };

    // 16 output channels. Output plane o from its finished accumulators:
    // lane (kgrp, row) holds channels 4 kgrp .. + 3 of voxel `row` of tile tt
    // (x-row wu + 4 tt). Both stores are always issued (outputs outside the
    // grid or before z0 go to the sink, 1 KB per work-group, 64 work-groups
    // apart).
    auto emit16 = [&](int o, const f32x4_t (&acc)[2]) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int gy = y0 + wu + ZW * tt, gxo = x0 + row;
            const bool ok = (o >= z0) & (gy < d.ny) & (gxo < d.nx);
            const size_t v = ok ? (size_t)((o * d.ny + gy) * d.nx) + gxo : 0;
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
            uint2* dst = ok ? reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + v * 16 + 4 * kgrp)
                            : static_cast<uint2*>(sink) + (blockIdx.x & 63) * 128 + 64 * tt + lane;
            *dst = make_uint2(pack_bf16x2(val[0], val[1]), pack_bf16x2(val[2], val[3]));
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
        const unsigned char* sb = slots + (p & 1) * PL::SLOT;
        if constexpr (CIN == 16) {
#pragma unroll
            for (int c = 0; c < ZP_PAIRS; ++c) {
                bf16x8_t a[2];
                frag16(sb, c, a);
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    nw[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[c], a[tt], nw[tt], 0, 0, 0);
                    md[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[ZP_PAIRS + c], a[tt], md[tt], 0, 0, 0);
                    dn[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[2 * ZP_PAIRS + c], a[tt], dn[tt], 0, 0, 0);
                }
            }
        } else {
            bf16x8_t a[2];
            frag2(sb, a);
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                nw[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[0], a[tt], nw[tt], 0, 0, 0);
                md[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[1], a[tt], md[tt], 0, 0, 0);
                dn[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[2], a[tt], dn[tt], 0, 0, 0);
            }
        }
        store_plane((p + 1) & 1, st);
        emit16(p - 1, dn);
        __syncthreads();
    };
    // One output channel: D = P W, lane (kgrp, row) holds voxels 4 kgrp .. + 3
    // of the tile in column `row`. Step q = p - z0 + 1 uses the weight
    // rotation R = q mod 3: column (R + 1) mod 3 takes dz = -1 (output p + 1),
    // column R dz = 0 (output p), column (R + 2) mod 3 dz = +1 (output
    // p - 1, complete after this step: stored, then cleared). (Stores to a
    // sink from every lane measured 2x slower here: the sink lines were
    // contended.)
    auto step1 = [&](int p, auto rot, PlaneRegs& ld, const PlaneRegs& st, f32x4_t (&acc)[2]) {
        constexpr int R = decltype(rot)::value;
        fetch_plane(p + 2, ld);
        const unsigned char* sb = slots + (p & 1) * PL::SLOT;
#pragma unroll
        for (int c = 0; c < ZP_PAIRS; ++c) {
            bf16x8_t a[2];
            frag16(sb, c, a);
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
                const int gy = y0 + wu + ZW * tt, gx = x0 + 4 * kgrp;
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
    // md = S[(q + 2) % 3], dn = S[(q + 1) % 3]. (A third register set, loads
    // two planes ahead, measured no faster.)
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
// layout of k_conv3d_z for input width CIN (2: one chunk per dz of the 9
// in-plane taps x 2 channels; 16: chunks of two in-plane taps of one dz, or
// with one output channel the B-operand column rotations; cin <= CIN,
// cout <= 16, missing entries zero). mirror: use W[26 - t][co][ci] (input
// gradient: mirrored taps, input and output channels swapped).
__global__ void k_swizzle_weights(const float* __restrict__ w, int cin, int cout, int CIN, int mirror,
                                  uint16_t* __restrict__ out) {
    const int nch = CIN == 16 ? ZPlane<16>::NCH : ZPlane<2>::NCH;
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
            // chunk dzi: (in-plane tap k / 2, channel k % 2) of plane dz = dzi - 1
            tap = k / 2 < 9 ? 9 * c + k / 2 : 27;
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

// Resident work-groups per CU of a kernel (cached per kernel).
int conv_blocks_per_cu(const void* f) {
    static const void* keys[32] = {};
    static int vals[32] = {};
    for (int i = 0; i < 32; ++i)
        if (keys[i] == f) return vals[i];
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, ZNT, 0) != hipSuccess || nb < 1) nb = 1;
    for (int i = 0; i < 32; ++i)
        if (!keys[i]) {
            vals[i] = nb;
            keys[i] = f;
            break;
        }
    return nb;
}

// One convolution layer through k_conv3d_z<MODE, CIN, TR>. The z chunk: when
// the footprints alone are fewer than the resident work-groups, z is split
// so the grid fills them once (at 128^3 with the 16-channel kernels: 128
// footprints x 6 chunks of 22 planes = 768 = 3 per CU); chunks stay within
// 4 .. 32 planes (each costs two extra input planes; at 64^3, 4-plane chunks
// measured 30 us per forward against 33 with an 8-plane floor).
template <int MODE, int CIN, typename TR>
hipError_t conv_z(const Dims& d, const void* in, const void* wsw, void* out, const void* mask, const double* scale_rms2,
                  double scale_mul, const void* zeros, void* sink, const TR* r, const float* g, const double* rr,
                  hipStream_t s) {
    if (d.nvox == 0) return hipSuccess;
    if (d.nvox > INT32_MAX) return hipErrorInvalidValue;  // 32-bit voxel offsets
    int ncu = 0;
    if (conv_device_cus(&ncu) != hipSuccess) return hipErrorInvalidDevice;
    const int nbx = (d.nx + CB_X - 1) / CB_X, nby = (d.ny + ZROWS - 1) / ZROWS;
    const int64_t fp = (int64_t)nbx * nby;
    const int64_t slots = (int64_t)conv_blocks_per_cu((const void*)k_conv3d_z<MODE, CIN, TR>) * ncu;
    const int64_t nzc = fp >= slots ? 1 : slots / fp;
    const int zc = (int)std::min<int64_t>(32, std::max<int64_t>(4, (d.nz + nzc - 1) / nzc));
    const int64_t nb = fp * ((d.nz + zc - 1) / zc);
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_conv3d_z<MODE, CIN, TR>), dim3((unsigned)nb), dim3(ZNT), 0, s, d, nbx, nby, zc,
                       static_cast<const uint16_t*>(in), static_cast<const uint16_t*>(wsw), out,
                       static_cast<const uint16_t*>(mask), scale_rms2, scale_mul, zeros, sink, r, g, rr);
    return hipGetLastError();
}

hipError_t launch_conv3d(int nx, int ny, int nz, int cin, int mode, const void* in, const void* wsw, void* out,
                         const void* mask, const double* scale_rms2, double scale_mul, const void* zeros, void* sink,
                         hipStream_t s) {
    const Dims d{nx, ny, nz, (int64_t)nx * ny * nz};
#define PCGMI_CONVZ(MO, CI) \
    conv_z<MO, CI, void>(d, in, wsw, out, mask, scale_rms2, scale_mul, zeros, sink, nullptr, nullptr, nullptr, s)
    if (cin == 16) {
        switch (mode) {
            case OUT_RELU_BF16: return PCGMI_CONVZ(OUT_RELU_BF16, 16);
            case OUT_SCALED_F32: return PCGMI_CONVZ(OUT_SCALED_F32, 16);
            case OUT_MASK_BF16: return PCGMI_CONVZ(OUT_MASK_BF16, 16);
            case OUT_LINEAR_BF16: return PCGMI_CONVZ(OUT_LINEAR_BF16, 16);
            default: return hipErrorInvalidValue;
        }
    } else if (cin == 2) {
        switch (mode) {
            case OUT_RELU_BF16: return PCGMI_CONVZ(OUT_RELU_BF16, 2);
            case OUT_MASK_BF16: return PCGMI_CONVZ(OUT_MASK_BF16, 2);
            case OUT_LINEAR_BF16: return PCGMI_CONVZ(OUT_LINEAR_BF16, 2);
            default: return hipErrorInvalidValue;  // one output channel follows a 16-channel layer only
        }
    }
#undef PCGMI_CONVZ
    return hipErrorInvalidValue;
}

// The first layer (2 -> 16, ReLU) straight from r (F32, F64 or BF16) and g.
hipError_t launch_conv3d_input(int nx, int ny, int nz, int dt, const void* r, const float* g, const double* rr,
                               const void* wsw, void* out, const void* zeros, void* sink, hipStream_t s) {
    const Dims d{nx, ny, nz, (int64_t)nx * ny * nz};
#define PCGMI_CONVIN(T) \
    conv_z<OUT_RELU_BF16, 2, T>(d, nullptr, wsw, out, nullptr, nullptr, 1.0, zeros, sink, static_cast<const T*>(r), g, \
                                rr, s)
    if (dt == DT_F32) return PCGMI_CONVIN(float);
    if (dt == DT_F64) return PCGMI_CONVIN(double);
    if (dt == DT_BF16) return PCGMI_CONVIN(bf16);
#undef PCGMI_CONVIN
    return hipErrorInvalidValue;
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

int conv_sink_bytes() { return CONV_SINK; }

int conv_swizzle_elems(int CIN) { return (CIN == 16 ? ZPlane<16>::NCH : ZPlane<2>::NCH) * 64 * 8; }

}  // namespace pcgmi
