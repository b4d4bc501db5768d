// common.hpp -- device-side building blocks shared by the gfx950 kernels:
// storage types and their conversions, 16-byte vector access, wavefront and
// work-group reductions, the last-work-group ("ticket") grid reduction and
// the XCD-aware block -> tile mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcgmi {

// ---------------------------------------------------------------------------
// Storage types. Vectors live in HBM as float, double, _Float16 or BF16 (raw
// 16-bit pattern). Arithmetic happens in the compute type C: float for the
// 32/16-bit types, double for double.
// ---------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};

template <typename T> struct Traits;
template <> struct Traits<float> {
    using C = float;
    static constexpr int W = 4;  // elements per 16-byte vector
};
template <> struct Traits<double> {
    using C = double;
    static constexpr int W = 2;
};
template <> struct Traits<_Float16> {
    using C = float;
    static constexpr int W = 8;
};
template <> struct Traits<bf16> {
    using C = float;
    static constexpr int W = 8;
};

// An FP32 value kept as FP32 for the conversion that follows: without the
// (empty) barrier the compiler merges an FP64 -> FP32 narrowing in front of
// a 16-bit conversion into a single FP64 -> 16-bit rounding, while the
// library rounds twice (FP64 -> FP32 -> 16 bits), as the oracle does.
__device__ __forceinline__ float keep_f32(float f) {
    __asm__("" : "+v"(f));
    return f;
}

// Round FP32 to BF16, nearest with ties to even; NaN stays a quiet NaN.
// gfx950 converts in hardware (v_cvt_pk_bf16_f32, two values per
// instruction; equal to the integer rounding on all 2^32 inputs); the integer
// form it replaces took five operations and a NaN test per value, which
// showed in the 16-bit direction kernel (the loader rounds p = D^-1 r +
// beta p_old to BF16 for the tile and its halo).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)keep_f32(f));
}

__device__ __forceinline__ float to_c(float v) { return v; }
__device__ __forceinline__ double to_c(double v) { return v; }
__device__ __forceinline__ float to_c(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_c(bf16 v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

template <typename T> __device__ __forceinline__ T from_c(typename Traits<T>::C v);
template <> __device__ __forceinline__ float from_c<float>(float v) { return v; }
template <> __device__ __forceinline__ double from_c<double>(double v) { return v; }
template <> __device__ __forceinline__ _Float16 from_c<_Float16>(float v) { return (_Float16)keep_f32(v); }
template <> __device__ __forceinline__ bf16 from_c<bf16>(float v) { return bf16{f32_to_bf16_bits(v)}; }

// Value after a round trip through the storage type (what a later load sees).
template <typename T> __device__ __forceinline__ typename Traits<T>::C stored(typename Traits<T>::C v) {
    return to_c(from_c<T>(v));
}

// 16-byte vector load/store of W = Traits<T>::W consecutive elements.
template <typename T> struct alignas(16) Vec16 {
    T e[Traits<T>::W];
};

template <typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, typename Traits<T>::C* out) {
    Vec16<T> v = *reinterpret_cast<const Vec16<T>*>(p);
#pragma unroll
    for (int i = 0; i < Traits<T>::W; ++i) out[i] = to_c(v.e[i]);
}

template <typename T>
__device__ __forceinline__ void store_vec(T* __restrict__ p, const typename Traits<T>::C* in) {
    Vec16<T> v;
#pragma unroll
    for (int i = 0; i < Traits<T>::W; ++i) v.e[i] = from_c<T>(in[i]);
    *reinterpret_cast<Vec16<T>*>(p) = v;
}

template <typename T>
__device__ __forceinline__ void load_vec_nt(const T* __restrict__ p, typename Traits<T>::C* out) {
    using U = __attribute__((__vector_size__(16))) unsigned int;
    U raw = __builtin_nontemporal_load(reinterpret_cast<const U*>(p));
    Vec16<T> v;
    __builtin_memcpy(&v, &raw, 16);
#pragma unroll
    for (int i = 0; i < Traits<T>::W; ++i) out[i] = to_c(v.e[i]);
}

template <typename T>
__device__ __forceinline__ void store_vec_nt(T* __restrict__ p, const typename Traits<T>::C* in) {
    using U = __attribute__((__vector_size__(16))) unsigned int;
    Vec16<T> v;
#pragma unroll
    for (int i = 0; i < Traits<T>::W; ++i) v.e[i] = from_c<T>(in[i]);
    U raw;
    __builtin_memcpy(&raw, &v, 16);
    __builtin_nontemporal_store(raw, reinterpret_cast<U*>(p));
}

// ---------------------------------------------------------------------------
// Reductions. Fixed butterfly order, so results are deterministic.
// ---------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename R> __device__ __forceinline__ R wave_max(R v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        R w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Combine NC doubles over the work-group: component c is summed, or maxed
// when bit c of MAXMASK is set. The result is valid in thread 0.
// scratch: at least NC * 16 doubles of LDS (up to 16 wavefronts).
template <int NC, unsigned MAXMASK>
__device__ __forceinline__ void block_reduce(double (&v)[NC], double* scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = ((MAXMASK >> c) & 1u) ? wave_max(v[c]) : wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) scratch[c * 16 + wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = scratch[c * 16];
            for (int w = 1; w < nw; ++w) {
                double t = scratch[c * 16 + w];
                if ((MAXMASK >> c) & 1u) s = t > s ? t : s;
                else s += t;
            }
            v[c] = s;
        }
    }
    __syncthreads();
}

// Grid reduction through per-work-group partials: every work-group stores its
// NC partials at partials[NC * g + c]; the last work-group to arrive (an
// atomic ticket, with release/acquire fences at agent scope so partials
// written on other XCDs are visible) combines all partials in index order in
// FP64 and returns true with the totals in tot (thread 0 only). The ticket
// counter is reset to zero for the next launch.
template <int NC, unsigned MAXMASK>
__device__ __forceinline__ bool grid_reduce(double (&v)[NC], double* __restrict__ partials,
                                            unsigned* ticket, unsigned nblocks, unsigned gid,
                                            double* lds, double (&tot)[NC]) {
    __shared__ int s_last;
    block_reduce<NC, MAXMASK>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            __hip_atomic_store(&partials[NC * gid + c], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned t = atomicAdd(ticket, 1u);
        s_last = (t == nblocks - 1);
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (unsigned i = threadIdx.x; i < nblocks; i += blockDim.x)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double t = __hip_atomic_load(&partials[NC * i + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((MAXMASK >> c) & 1u) acc[c] = t > acc[c] ? t : acc[c];
            else acc[c] += t;
        }
    block_reduce<NC, MAXMASK>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) tot[c] = acc[c];
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

// ---------------------------------------------------------------------------
// XCD-aware mapping. The dispatcher hands work-group b to XCD (b mod 8); this
// bijection gives each XCD a contiguous range of logical tiles so that tiles
// sharing halo data share an L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nblocks) {
    const unsigned nx = 8;
    unsigned q = nblocks / nx, rem = nblocks % nx;
    unsigned x = b % nx, j = b / nx;
    unsigned start = x * q + (x < rem ? x : rem);
    return start + j;
}

}  // namespace pcgmi
