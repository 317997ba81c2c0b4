// patch_smooth_noalloc: patch_smooth whose per-call scratch (the residual
// vector of the colour loop and the two CG counters) lives in a file-scope
// device array instead of the caller's workspace, for callers that cannot
// allocate device memory at the call site (HIP graph capture, tight serving
// loops).  The array is per device and is looked up with hipGetSymbolAddress
// on the first call on that device; host code never uses its name as an
// address.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "handle.hpp"
#include "mg_kernels.hpp"
#include "mlp.hpp"

namespace {

constexpr size_t kCounterBytes = 256;   // two 64-bit CG counters, padded to keep the vector 256-byte aligned

__device__ __align__(256) unsigned char scratch[STOKESMG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (looked up once per device)
hipError_t scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int stokesmg_noalloc_scratch_size(size_t* bytes) {
    if (!bytes) return STOKESMG_EINVAL;
    *bytes = STOKESMG_NOALLOC_SCRATCH_BYTES;
    return STOKESMG_OK;
}

int patch_smooth_noalloc(stokesmg_t* h, int level, int dtype, void* x, const void* b, int n_sweeps,
                         int64_t* cg_iterations, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (level < 0 || level >= h->n_levels) return h->fail(STOKESMG_EINVAL, "level out of range");
    if (dtype != STOKESMG_F64 && dtype != STOKESMG_F32) return h->fail(STOKESMG_EINVAL, "dtype must be F64 or F32");
    if (!h->ws) return h->fail(STOKESMG_ENOMEM, "no workspace set (it holds the level tables)");
    if (!x || !b || n_sweeps < 0) return h->fail(STOKESMG_EINVAL, "null vector or negative sweep count");
    if (h->lv[level].n < 2) return h->fail(STOKESMG_EINVAL, "level has no interior vertex (n < 2)");
    const size_t es = dtype == STOKESMG_F64 ? 8 : 4;
    const size_t N = size_t(level_total(h, level));
    const size_t bytes = N * es;
    if (kCounterBytes + bytes > STOKESMG_NOALLOC_SCRATCH_BYTES)
        return h->fail(STOKESMG_EINVAL, "level too large for the static scratch of patch_smooth_noalloc "
                                        "(one level vector + 256 bytes must fit STOKESMG_NOALLOC_SCRATCH_BYTES)");
    if (ranges_overlap(x, bytes, b, bytes) || ranges_overlap(x, bytes, h->ws, h->ws_bytes) ||
        ranges_overlap(b, bytes, h->ws, h->ws_bytes))
        return h->fail(STOKESMG_EINVAL, "x, b and the workspace must not overlap");
    void* base = nullptr;
    SMG_HIP(h, scratch_ptr(&base));
    unsigned long long* counters = static_cast<unsigned long long*>(base);
    void* r = static_cast<unsigned char*>(base) + kCounterBytes;
    if (ranges_overlap(x, bytes, base, STOKESMG_NOALLOC_SCRATCH_BYTES) ||
        ranges_overlap(b, bytes, base, STOKESMG_NOALLOC_SCRATCH_BYTES))
        return h->fail(STOKESMG_EINVAL, "x and b must not lie in the library's scratch");
    const bool f64 = dtype == STOKESMG_F64;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the counters start at zero on every call (a fill kernel: safe under graph capture)
    SMG_HIP(h, smg::launch_zero(true, counters, 2, st));
    for (int s = 0; s < n_sweeps; ++s)
        if (int rc = smg::smooth_sweep(h, level, f64, x, b, st, nullptr, r, counters, true)) return rc;
    if (cg_iterations) {
        unsigned long long c[2] = {0, 0};
        SMG_HIP(h, hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, st));
        SMG_HIP(h, hipStreamSynchronize(st));
        *cg_iterations = int64_t(c[0]);
    }
    return STOKESMG_OK;
}

}  // extern "C"
