// noalloc.hip -- dot_noalloc: the dot product of dot / dot_f64 without a
// context and without any allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// dot runs two kernels: k_dot writes one FP64 partial per work-group into the
// context's workspace, and k_dot_finish sums them in index order. Here the
// partials live in a file-scope device array instead. Host code never passes
// the array's name to a kernel (in host code it is a host-side stand-in, not a
// device address): the first call on each device looks up the array's device
// address with hipGetSymbolAddress, with that device current, and keeps it per
// device; every later use goes through that address.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "internal.hpp"
#include "pcgmi.h"

namespace pcgmi {
const char* set_error(pcg_status st, const char* msg);
}

using namespace pcgmi;

namespace {

// The dot launcher caps its grid at 1024 work-groups, one FP64 partial each.
constexpr size_t NOALLOC_PARTIALS = 1024;

static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {};  // device address of `scratch` per device, 0 until looked up

pcg_status nerr(pcg_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pcg_status nerr(pcg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_error(st, buf);
    return st;
}

// Device address of `scratch` on the current device (looked up once per device).
pcg_status scratch_of_current_device(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return nerr(PCG_E_HIP, "dot_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return nerr(PCG_E_UNSUPPORTED, "dot_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return nerr(PCG_E_HIP, "dot_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return PCG_OK;
}

}  // namespace

extern "C" pcg_status dot_noalloc(pcg_dtype storage, int64_t n, const void* x, const void* y, float* out_f32,
                                  double* out_f64, void* hip_stream) {
    if (storage < PCG_F32 || storage > PCG_F64) return nerr(PCG_E_ARG, "dot_noalloc: unknown storage type %d", (int)storage);
    if (n < 0) return nerr(PCG_E_ARG, "dot_noalloc: negative length");
    if (n > PCG_DOT_NOALLOC_MAX_N) return nerr(PCG_E_ARG, "dot_noalloc: length %lld above the maximum 2^40", (long long)n);
    if (!out_f32 && !out_f64) return nerr(PCG_E_ARG, "dot_noalloc: null output");
    if (n > 0 && (!x || !y)) return nerr(PCG_E_ARG, "dot_noalloc: null pointer");
    if (n > 0 && (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u) != 0))
        return nerr(PCG_E_ARG, "dot_noalloc: pointers must be 16-byte aligned");
    double* part = nullptr;
    const pcg_status st = scratch_of_current_device(&part);
    if (st != PCG_OK) return st;
    // the partials of every launch are written before they are read: nothing to clear
    const Red red{part, nullptr, NOALLOC_PARTIALS};
    const hipError_t e = launch_dot((int)storage, n, x, y, out_f32, out_f64, red, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return nerr(PCG_E_HIP, "dot_noalloc: launch failed: %s", hipGetErrorString(e));
    return PCG_OK;
}
