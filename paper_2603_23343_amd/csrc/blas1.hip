// blas1.hip -- streaming kernels: axpy (paper Sec. IV's element-wise update),
// dot (Sec. V's global reduction), the zero-guess start of a solve, fills and
// type conversions.
//
// Each thread moves 16-byte vectors (4 FP32, 8 BF16/FP16, 2 FP64 elements);
// consecutive threads touch consecutive vectors, so every wavefront access
// is one contiguous 1 KiB segment. axpy and dot stream with non-temporal
// loads and stores: their vectors are touched once, and keeping them out of
// L2 and the last-level cache measured faster at 512^3. The dot keeps one accumulator per vector
// lane in the compute type, reduces across the wavefront with a fixed
// butterfly and across work-groups with the last-work-group ticket, so the
// result is deterministic.
#include "ops.hpp"
#include "zkernel.hpp"

namespace pcgmi {

namespace {

constexpr int NT = STREAM_THREADS;
constexpr int AXPY_UNROLL = 4;

template <typename T>
__global__ void __launch_bounds__(NT) k_axpy(int64_t n, typename Traits<T>::C alpha, const T* x, const T* y, T* z) {
    using C = typename Traits<T>::C;
    constexpr int W = Traits<T>::W;
    const int64_t nvec = n / W;
    const int64_t base = (int64_t)blockIdx.x * NT * AXPY_UNROLL + threadIdx.x;
    C xv[AXPY_UNROLL][W], yv[AXPY_UNROLL][W];
#pragma unroll
    for (int u = 0; u < AXPY_UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * NT;
        if (i < nvec) {
            load_vec_nt<T>(x + i * W, xv[u]);
            load_vec_nt<T>(y + i * W, yv[u]);
        }
    }
    const C a = alpha;
#pragma unroll
    for (int u = 0; u < AXPY_UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * NT;
        if (i < nvec) {
            C zv[W];
#pragma unroll
            for (int e = 0; e < W; ++e) zv[e] = a * xv[u][e] + yv[u][e];
            store_vec_nt<T>(z + i * W, zv);
        }
    }
    // Ragged tail (fewer than W elements): block 0.
    if (blockIdx.x == 0) {
        const int64_t t = nvec * W + threadIdx.x;
        if (t < n) z[t] = from_c<T>(a * to_c(x[t]) + to_c(y[t]));
    }
}

template <typename T>
__global__ void __launch_bounds__(NT) k_dot(int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                                            float* out_f32, double* out_f64, Red red) {
    using C = typename Traits<T>::C;
    constexpr int W = Traits<T>::W;
    __shared__ double scratch[16];
    const int64_t nvec = n / W;
    C acc[W];
#pragma unroll
    for (int e = 0; e < W; ++e) acc[e] = C(0);
    // Work-group b streams its own contiguous range of vectors, four vector
    // pairs in flight per thread, with non-temporal loads (nothing is re-read:
    // keeping the lines out of the caches measured 6.1 -> 7.0 TB/s at 512^3,
    // against 5.4 TB/s for a grid-stride walk).
    const int64_t per = (nvec + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < nvec ? lo + per : nvec;
    constexpr int U = 4;
    int64_t i = lo + threadIdx.x;
    for (; i + (U - 1) * NT < hi; i += U * NT) {
        C a[U][W], b[U][W];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            load_vec_nt<T>(x + (i + u * NT) * W, a[u]);
            load_vec_nt<T>(y + (i + u * NT) * W, b[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < W; ++e) acc[e] += a[u][e] * b[u][e];
    }
    for (; i < hi; i += NT) {
        C a[W], b[W];
        load_vec_nt<T>(x + i * W, a);
        load_vec_nt<T>(y + i * W, b);
#pragma unroll
        for (int e = 0; e < W; ++e) acc[e] += a[e] * b[e];
    }
    if (blockIdx.x == 0) {
        const int64_t t = nvec * W + threadIdx.x;
        if (t < n) acc[0] += to_c(x[t]) * to_c(y[t]);
    }
    double v[1] = {0.0};
#pragma unroll
    for (int e = 0; e < W; ++e) v[0] += (double)acc[e];
    // partial per work-group; k_dot_finish sums them in index order (a
    // kernel boundary instead of a release fence per work-group)
    block_reduce<1, 0u>(v, scratch);
    if (threadIdx.x == 0) red.partials[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(NT) k_dot_finish(const double* __restrict__ partials, unsigned nblocks,
                                                   float* out_f32, double* out_f64) {
    __shared__ double scratch[16];
    double v[1] = {0.0};
    for (unsigned i = threadIdx.x; i < nblocks; i += NT) v[0] += partials[i];
    block_reduce<1, 0u>(v, scratch);
    if (threadIdx.x == 0) {
        if (out_f32) *out_f32 = (float)v[0];
        if (out_f64) *out_f64 = v[0];
    }
}

// Start of a solve from x0 = 0: r = b, x = 0, p0 = 0 (the first direction
// kernel reads p0 as p_old with beta = 0; p1 is written before it is read)
// and the totals {b.b, b.b, sum dinv b^2} for the solve state.
template <typename T, typename X>
__global__ void __launch_bounds__(NT) k_start_zero(int64_t n, const T* __restrict__ b, T* __restrict__ r,
                                                   X* __restrict__ x, T* __restrict__ p0,
                                                   const T* __restrict__ dinv, SolveState* st, double* hist,
                                                   Red red) {
    using C = typename Traits<T>::C;
    constexpr int W = Traits<T>::W;
    __shared__ double scratch[48];
    const int64_t nvec = n / W;
    const int64_t stride = (int64_t)gridDim.x * NT;
    const C dconst = (C)st->dinv;
    C acc = C(0), accz = C(0);
    C zero[W];
    double xz[W];
#pragma unroll
    for (int e = 0; e < W; ++e) {
        zero[e] = C(0);
        xz[e] = 0.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nvec; i += stride) {
        C a[W], d[W];
        load_vec<T>(b + i * W, a);
        if (dinv) load_vec<T>(dinv + i * W, d);
        store_vec<T>(r + i * W, a);
        store_vec<T>(p0 + i * W, zero);
        st_any<X, W>(x, i * W, xz);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            acc += a[e] * a[e];
            accz += (dinv ? d[e] : dconst) * a[e] * a[e];
        }
    }
    if (blockIdx.x == 0) {
        const int64_t t = nvec * W + threadIdx.x;
        if (t < n) {
            C a = to_c(b[t]);
            r[t] = b[t];
            p0[t] = from_c<T>(C(0));
            x[t] = from_c<X>((typename Traits<X>::C)0);
            acc += a * a;
            accz += (dinv ? to_c(dinv[t]) : dconst) * a * a;
        }
    }
    // partials per work-group; k_zfinish applies FinStart (a kernel boundary
    // instead of an agent-scope release fence per work-group: 226 us at 256^3
    // with 2048 work-groups before)
    double v[3] = {(double)acc, (double)acc, (double)accz};
    block_reduce<3, 0u>(v, scratch);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) red.partials[3 * blockIdx.x + c] = v[c];
}

__global__ void __launch_bounds__(NT) k_zero_bytes(int64_t nbytes, unsigned char* p) {
    const int64_t nvec = nbytes / 16;
    const int64_t stride = (int64_t)gridDim.x * NT;
    using U = __attribute__((__vector_size__(16))) unsigned int;
    U z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nvec; i += stride)
        reinterpret_cast<U*>(p)[i] = z;
    if (blockIdx.x == 0) {
        const int64_t t = nvec * 16 + threadIdx.x;
        if (t < nbytes) p[t] = 0;
    }
}

// dst = src through the compute type of the wider side: FP64 -> FP32 -> 16-bit
// when narrowing from double to a 16-bit type (two roundings to nearest even).
template <typename S, typename D>
__global__ void __launch_bounds__(NT) k_convert(int64_t n, const S* __restrict__ src, D* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        double v = (double)to_c(src[i]);
        dst[i] = from_c<D>((typename Traits<D>::C)v);
    }
}

inline unsigned stream_blocks(int64_t nvec, int64_t per_block, int64_t cap) {
    int64_t b = (nvec + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_axpy(int dt, int64_t n, double alpha, const void* x, const void* y, void* z, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        const int64_t nvec = n / Traits<T>::W;
        const unsigned nb = stream_blocks(nvec, (int64_t)NT * AXPY_UNROLL, INT32_MAX);
        // alpha in the arithmetic type: FP32 for 32- and 16-bit storage, FP64 for FP64
        const typename Traits<T>::C a = (typename Traits<T>::C)alpha;
        hipLaunchKernelGGL(k_axpy<T>, dim3(nb), dim3(NT), 0, s, n, a, static_cast<const T*>(x),
                           static_cast<const T*>(y), static_cast<T*>(z));
        return hipGetLastError();
    });
}

hipError_t launch_dot(int dt, int64_t n, const void* x, const void* y, float* out_f32, double* out_f64, Red red,
                      hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        const int64_t nvec = n / Traits<T>::W;
        // 1024 work-groups (4 per CU) streamed best in a sweep of 1024..16384
        const unsigned nb = stream_blocks(nvec, (int64_t)NT * 4, 1024);
        if ((size_t)nb > red.cap) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_dot<T>, dim3(nb), dim3(NT), 0, s, n, static_cast<const T*>(x),
                           static_cast<const T*>(y), out_f32, out_f64, red);
        hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(NT), 0, s, red.partials, nb, out_f32, out_f64);
        return hipGetLastError();
    });
}

hipError_t launch_pcg_start_zero(int dt, int64_t n, const void* b, void* r, void* x, int xdt, void* p0,
                                 const void* dinv, SolveState* st, double* hist, Red red, hipStream_t s) {
    return dispatch_dt(dt, [&](auto tag) {
        using T = decltype(tag);
        const int64_t nvec = n / Traits<T>::W;
        const unsigned nb = stream_blocks(nvec, (int64_t)NT * 4, DOT_MAX_BLOCKS);
        if ((size_t)3 * nb > red.cap) return hipErrorInvalidValue;
        auto go = [&](auto xtag) {
            using X = decltype(xtag);
            hipLaunchKernelGGL((k_start_zero<T, X>), dim3(nb), dim3(NT), 0, s, n, static_cast<const T*>(b),
                               static_cast<T*>(r), static_cast<X*>(x), static_cast<T*>(p0),
                               static_cast<const T*>(dinv), st, hist, red);
            hipLaunchKernelGGL((k_zfinish<3, 0u, FinStart>), dim3(1), dim3(NT), 0, s, red.partials, nb,
                               FinStart{st, hist}, nullptr);
            return hipGetLastError();
        };
        if (xdt == DT_F64) return go(double{});
        if (xdt == DT_F32) return go(float{});
        if (xdt == dt) return go(T{});
        return hipErrorInvalidValue;
    });
}

hipError_t launch_zero(int dt, int64_t n, void* p, hipStream_t s) {
    const int64_t nbytes = n * (int64_t)dt_size(dt);
    if (nbytes <= 0) return hipSuccess;
    const unsigned nb = stream_blocks(nbytes / 16, (int64_t)NT * 4, 4096);
    hipLaunchKernelGGL(k_zero_bytes, dim3(nb), dim3(NT), 0, s, nbytes, static_cast<unsigned char*>(p));
    return hipGetLastError();
}

hipError_t launch_convert(int sdt, int ddt, int64_t n, const void* src, void* dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return dispatch_dt(sdt, [&](auto stag) {
        using S = decltype(stag);
        return dispatch_dt(ddt, [&](auto dtag) {
            using D = decltype(dtag);
            const unsigned nb = stream_blocks(n, (int64_t)NT * 4, 8192);
            hipLaunchKernelGGL((k_convert<S, D>), dim3(nb), dim3(NT), 0, s, n, static_cast<const S*>(src),
                               static_cast<D*>(dst));
            return hipGetLastError();
        });
    });
}

}  // namespace pcgmi
