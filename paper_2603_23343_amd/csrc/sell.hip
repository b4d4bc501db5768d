// sell.hip -- SpMV of a general sparse matrix in sliced ELLPACK
// (SELL-C-sigma; Kreutzer, Hager, Wellein, Fehske, Bishop, SIAM J. Sci.
// Comput. 36(5), 2014), the storage of the GPU comparison system of the
// paper's Sec. VII-A, whose CG is built from norm, dot, axpy and SpMV.
//
// The layout is built on the host from compressed rows. On the device one
// wavefront owns one chunk of C = 64 rows, one lane per row: slot j of the
// chunk is a contiguous 256-byte run of column indices and one of values, so
// both streams load fully coalesced (non-temporal: each slot is read once per
// product), and the x gathers go through L2. The work-group -> chunk mapping
// is XCD-aware: each XCD walks a contiguous range of rows, so the x lines a
// row's neighbours share (for a grid operator, the planes above and below)
// stay in that XCD's L2.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "pcgmi.h"

namespace pcgmi {
const char* set_error(pcg_status st, const char* msg);
}

using namespace pcgmi;

struct pcg_sell_s {
    int64_t nrows = 0, ncols = 0, nnz = 0, nchunks = 0, nslots = 0;
    int64_t* chunk_ptr = nullptr;  // device, nchunks + 1
    int32_t* col = nullptr;        // device, nslots
    float* val = nullptr;          // device, nslots
    int32_t* perm = nullptr;       // device, nrows (null when sigma = 1)
    hipStream_t stream = nullptr;
};

namespace {

constexpr int SELL_C = 64;       // rows per chunk = wavefront width
constexpr int SELL_WAVES = 4;    // chunks per work-group
constexpr int SELL_UNROLL = 8;   // slots in flight per lane

pcg_status serr(pcg_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pcg_status serr(pcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(st, buf);
    return st;
}

template <bool PERM>
__global__ void __launch_bounds__(SELL_C * SELL_WAVES)
    k_sell_spmv(int64_t nrows, int64_t nchunks, const int64_t* __restrict__ chunk_ptr,
                const int32_t* __restrict__ col, const float* __restrict__ val, const int32_t* __restrict__ perm,
                const float* __restrict__ x, float* __restrict__ y) {
    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t c = (int64_t)b * SELL_WAVES + (threadIdx.x >> 6);
    if (c >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const int64_t base = chunk_ptr[c];
    const int w = (int)((chunk_ptr[c + 1] - base) / SELL_C);
    const int32_t* cp = col + base + lane;
    const float* vp = val + base + lane;
    float acc = 0.0f;
    for (int j = 0; j < w; j += SELL_UNROLL) {
        int ci[SELL_UNROLL];
        float vi[SELL_UNROLL], xv[SELL_UNROLL];
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) {
            ci[u] = -1;
            vi[u] = 0.0f;
            if (j + u < w) {
                ci[u] = __builtin_nontemporal_load(cp + (int64_t)(j + u) * SELL_C);
                vi[u] = __builtin_nontemporal_load(vp + (int64_t)(j + u) * SELL_C);
            }
        }
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u) xv[u] = ci[u] >= 0 ? x[ci[u]] : 0.0f;
        // entries in storage order; padding (column -1) is skipped
#pragma unroll
        for (int u = 0; u < SELL_UNROLL; ++u)
            if (ci[u] >= 0) acc = __builtin_fmaf(vi[u], xv[u], acc);
    }
    const int64_t s = c * SELL_C + lane;
    if (s < nrows) {
        const int64_t dst = PERM ? (int64_t)perm[s] : s;
        __builtin_nontemporal_store(acc, y + dst);
    }
}

}  // namespace

extern "C" {

pcg_status pcg_sell_build(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                          const float* values, int chunk, int sigma, int64_t* nchunks, int64_t* nslots,
                          int64_t* chunk_ptr, int32_t* perm, int32_t* col_out, float* val_out) {
    const int64_t IMAX = 2147483647;
    if (nrows < 0 || nrows > IMAX || ncols < 0 || ncols > IMAX)
        return serr(PCG_E_ARG, "pcg_sell_build: nrows and ncols must be in [0, 2^31 - 1]");
    if (chunk < 1 || sigma < 1 || (sigma > 1 && sigma % chunk != 0))
        return serr(PCG_E_ARG, "pcg_sell_build: chunk >= 1 and sigma = 1 or a multiple of chunk (got %d, %d)",
                    chunk, sigma);
    if (!nchunks || !nslots) return serr(PCG_E_ARG, "pcg_sell_build: null nchunks or nslots");
    if (!rowptr || (nrows > 0 && rowptr[nrows] > 0 && (!colidx || !values)))
        return serr(PCG_E_ARG, "pcg_sell_build: null compressed-row array");
    if (rowptr[0] != 0) return serr(PCG_E_ARG, "pcg_sell_build: rowptr[0] must be 0");
    for (int64_t i = 0; i < nrows; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return serr(PCG_E_ARG, "pcg_sell_build: rowptr decreases at row %lld", (long long)i);
    const int64_t nnz = rowptr[nrows];
    for (int64_t k = 0; k < nnz; ++k)
        if (colidx[k] < 0 || colidx[k] >= ncols)
            return serr(PCG_E_ARG, "pcg_sell_build: column %d of entry %lld out of range", colidx[k], (long long)k);

    // Sorted order: decreasing length inside each window of sigma rows.
    std::vector<int32_t> order((size_t)nrows);
    std::iota(order.begin(), order.end(), 0);
    if (sigma > 1)
        for (int64_t w0 = 0; w0 < nrows; w0 += sigma) {
            const int64_t w1 = std::min<int64_t>(w0 + sigma, nrows);
            std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int32_t a, int32_t b) {
                return rowptr[a + 1] - rowptr[a] > rowptr[b + 1] - rowptr[b];
            });
        }
    const int64_t nch = (nrows + chunk - 1) / chunk;
    int64_t slots = 0;
    std::vector<int64_t> cptr((size_t)nch + 1);
    for (int64_t c = 0; c < nch; ++c) {
        cptr[c] = slots;
        int64_t w = 0;
        for (int64_t s = c * chunk; s < std::min<int64_t>((c + 1) * chunk, nrows); ++s) {
            const int32_t r = order[s];
            w = std::max<int64_t>(w, rowptr[r + 1] - rowptr[r]);
        }
        slots += w * chunk;
    }
    cptr[nch] = slots;
    *nchunks = nch;
    *nslots = slots;
    if (!chunk_ptr && !perm && !col_out && !val_out) return PCG_OK;
    if (!chunk_ptr || (nrows > 0 && !perm) || (slots > 0 && (!col_out || !val_out)))
        return serr(PCG_E_ARG, "pcg_sell_build: output arrays must all be given");
    std::memcpy(chunk_ptr, cptr.data(), sizeof(int64_t) * (size_t)(nch + 1));
    if (nrows) std::memcpy(perm, order.data(), sizeof(int32_t) * (size_t)nrows);
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t w = (cptr[c + 1] - cptr[c]) / chunk;
        for (int64_t l = 0; l < chunk; ++l) {
            const int64_t s = c * chunk + l;
            const int64_t len = s < nrows ? rowptr[order[s] + 1] - rowptr[order[s]] : 0;
            const int64_t k0 = s < nrows ? rowptr[order[s]] : 0;
            for (int64_t j = 0; j < w; ++j) {
                const int64_t slot = cptr[c] + j * chunk + l;
                col_out[slot] = j < len ? colidx[k0 + j] : -1;
                val_out[slot] = j < len ? values[k0 + j] : 0.0f;
            }
        }
    }
    return PCG_OK;
}

pcg_status pcg_sell_destroy(pcg_sell A) {
    if (!A) return PCG_OK;
    (void)hipFree(A->chunk_ptr);
    (void)hipFree(A->col);
    (void)hipFree(A->val);
    (void)hipFree(A->perm);
    delete A;
    return PCG_OK;
}

pcg_status pcg_sell_create(pcg_sell* out, int64_t nrows, int64_t ncols, const int64_t* rowptr,
                           const int32_t* colidx, const float* values, int sigma, void* hip_stream) {
    if (!out) return serr(PCG_E_ARG, "pcg_sell_create: null output handle");
    *out = nullptr;
    int64_t nch = 0, slots = 0;
    pcg_status st = pcg_sell_build(nrows, ncols, rowptr, colidx, values, SELL_C, sigma, &nch, &slots, nullptr,
                                   nullptr, nullptr, nullptr);
    if (st != PCG_OK) return st;
    std::vector<int64_t> cptr((size_t)nch + 1);
    std::vector<int32_t> perm((size_t)nrows), col((size_t)slots);
    std::vector<float> val((size_t)slots);
    st = pcg_sell_build(nrows, ncols, rowptr, colidx, values, SELL_C, sigma, &nch, &slots, cptr.data(),
                        perm.data(), col.data(), val.data());
    if (st != PCG_OK) return st;
    auto* A = new (std::nothrow) pcg_sell_s;
    if (!A) return serr(PCG_E_NOMEM, "pcg_sell_create: out of host memory");
    A->nrows = nrows;
    A->ncols = ncols;
    A->nnz = rowptr[nrows];
    A->nchunks = nch;
    A->nslots = slots;
    A->stream = (hipStream_t)hip_stream;
    auto alloc = [&](void** p, size_t bytes) -> hipError_t { return bytes ? hipMalloc(p, bytes) : hipSuccess; };
    hipError_t e = alloc((void**)&A->chunk_ptr, sizeof(int64_t) * (size_t)(nch + 1));
    if (e == hipSuccess) e = alloc((void**)&A->col, sizeof(int32_t) * (size_t)slots);
    if (e == hipSuccess) e = alloc((void**)&A->val, sizeof(float) * (size_t)slots);
    if (e == hipSuccess && sigma > 1) e = alloc((void**)&A->perm, sizeof(int32_t) * (size_t)nrows);
    if (e == hipSuccess)
        e = hipMemcpy(A->chunk_ptr, cptr.data(), sizeof(int64_t) * (size_t)(nch + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && slots) e = hipMemcpy(A->col, col.data(), sizeof(int32_t) * (size_t)slots, hipMemcpyHostToDevice);
    if (e == hipSuccess && slots) e = hipMemcpy(A->val, val.data(), sizeof(float) * (size_t)slots, hipMemcpyHostToDevice);
    if (e == hipSuccess && A->perm)
        e = hipMemcpy(A->perm, perm.data(), sizeof(int32_t) * (size_t)nrows, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pcg_sell_destroy(A);
        return serr(e == hipErrorOutOfMemory ? PCG_E_NOMEM : PCG_E_HIP, "pcg_sell_create: %s", hipGetErrorString(e));
    }
    *out = A;
    return PCG_OK;
}

pcg_status pcg_sell_info(pcg_sell A, int64_t* nnz, int64_t* nslots, int64_t* nchunks) {
    if (!A) return serr(PCG_E_ARG, "pcg_sell_info: null handle");
    if (nnz) *nnz = A->nnz;
    if (nslots) *nslots = A->nslots;
    if (nchunks) *nchunks = A->nchunks;
    return PCG_OK;
}

pcg_status pcg_sell_spmv(pcg_sell A, const float* x, float* y) {
    if (!A) return serr(PCG_E_ARG, "pcg_sell_spmv: null handle");
    if (A->nrows == 0) return PCG_OK;
    if (!y || (A->ncols > 0 && !x)) return serr(PCG_E_ARG, "pcg_sell_spmv: null pointer");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 3u)
        return serr(PCG_E_ARG, "pcg_sell_spmv: x and y must be 4-byte aligned");
    const auto xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    const uintptr_t xb = (uintptr_t)A->ncols * 4, yb = (uintptr_t)A->nrows * 4;
    if (xb > 0 && xa < ya + yb && ya < xa + xb) return serr(PCG_E_ARG, "pcg_sell_spmv: x and y overlap");
    const int64_t blocks = (A->nchunks + SELL_WAVES - 1) / SELL_WAVES;
    const dim3 grid((unsigned)blocks), block(SELL_C * SELL_WAVES);
    if (A->perm)
        hipLaunchKernelGGL(k_sell_spmv<true>, grid, block, 0, A->stream, A->nrows, A->nchunks, A->chunk_ptr, A->col,
                           A->val, A->perm, x, y);
    else
        hipLaunchKernelGGL(k_sell_spmv<false>, grid, block, 0, A->stream, A->nrows, A->nchunks, A->chunk_ptr, A->col,
                           A->val, A->perm, x, y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return serr(PCG_E_HIP, "pcg_sell_spmv: launch failed: %s", hipGetErrorString(e));
    return PCG_OK;
}

}  // extern "C"
