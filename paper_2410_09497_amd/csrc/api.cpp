// C ABI of libstokesmg (include/stokesmg.h): handle, workspace, operator.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "apply.hpp"
#include "handle.hpp"
#include "stencil_tables.hpp"

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int64_t level_total(const stokesmg* h, int level) {
    const int64_t N1 = h->lv[level].N1;
    return 3 * (N1 - 1) * N1 * N1 + N1 * N1 * N1;
}

int check_level_dtype(stokesmg* h, int level, int dtype) {
    if (level < 0 || level >= h->n_levels) return h->fail(STOKESMG_EINVAL, "level out of range");
    if (dtype != STOKESMG_F64 && dtype != STOKESMG_F32) return h->fail(STOKESMG_EINVAL, "dtype must be F64 or F32");
    if (!h->ws) return h->fail(STOKESMG_ENOMEM, "no workspace set");
    return STOKESMG_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
    auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + bytes && pb < pa + bytes;
}

}  // namespace

extern "C" {

int stokesmg_create(const stokesmg_config* cfg, stokesmg_t** out) {
    if (!cfg || !out) return STOKESMG_EINVAL;
    *out = nullptr;
    const int n = cfg->n_cells, k = cfg->k, L = cfg->n_levels;
    if (n < 1 || (n & (n - 1)) != 0 || k < 1 || k > 5 || L < 1 || (n >> (L - 1)) < 1 ||
        ((n >> (L - 1)) << (L - 1)) != n || !(cfg->penalty_factor > 0))
        return STOKESMG_EINVAL;
    stokesmg* h = new (std::nothrow) stokesmg;
    if (!h) return STOKESMG_ENOMEM;
    h->cfg = *cfg;
    h->n_levels = L;
    try {
        smg::Ref1D ref(k);
        for (int l = 0; l < L; ++l) h->lv.push_back(smg::build_level_tables(ref, n >> (L - 1 - l), cfg->penalty_factor));
    } catch (const std::exception& e) {
        delete h;
        return STOKESMG_EINVAL;
    }
    size_t off = 0;
    const size_t tsz = smg::tab_size(k);
    for (int l = 0; l < L; ++l) {
        h->tab_f64.push_back(off);
        off = align256(off + tsz * sizeof(double));
        h->tab_f32.push_back(off);
        off = align256(off + tsz * sizeof(float));
    }
    h->ws_needed = off;
    *out = h;
    return STOKESMG_OK;
}

void stokesmg_destroy(stokesmg_t* h) { delete h; }

const char* stokesmg_last_error(const stokesmg_t* h) { return h ? h->err.c_str() : "null handle"; }

int stokesmg_num_levels(const stokesmg_t* h) { return h ? h->n_levels : STOKESMG_EINVAL; }

int stokesmg_sizes(const stokesmg_t* h, int level, int64_t* n_u_comp, int64_t* n_p, int64_t* n_total) {
    if (!h || level < 0 || level >= h->n_levels) return STOKESMG_EINVAL;
    const int64_t N1 = h->lv[level].N1;
    if (n_u_comp) *n_u_comp = (N1 - 1) * N1 * N1;
    if (n_p) *n_p = N1 * N1 * N1;
    if (n_total) *n_total = 3 * (N1 - 1) * N1 * N1 + N1 * N1 * N1;
    return STOKESMG_OK;
}

int stokesmg_workspace_size(const stokesmg_t* h, size_t* bytes) {
    if (!h || !bytes) return STOKESMG_EINVAL;
    *bytes = h->ws_needed;
    return STOKESMG_OK;
}

int stokesmg_set_workspace(stokesmg_t* h, void* dev_ptr, size_t bytes, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0)
        return h->fail(STOKESMG_EINVAL, "workspace must be a non-null, 256-byte aligned device pointer");
    if (bytes < h->ws_needed) return h->fail(STOKESMG_ENOMEM, "workspace smaller than stokesmg_workspace_size()");
    h->ws = static_cast<char*>(dev_ptr);
    h->ws_bytes = bytes;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t tsz = smg::tab_size(h->cfg.k);
    for (int l = 0; l < h->n_levels; ++l) {
        const auto& t = h->lv[l].stencil;
        std::vector<float> tf(t.begin(), t.end());
        SMG_HIP(h, hipMemcpyAsync(h->ws + h->tab_f64[l], t.data(), tsz * sizeof(double), hipMemcpyHostToDevice, st));
        SMG_HIP(h, hipMemcpyAsync(h->ws + h->tab_f32[l], tf.data(), tsz * sizeof(float), hipMemcpyHostToDevice, st));
        // the host buffers die at scope exit: finish the copies first
        SMG_HIP(h, hipStreamSynchronize(st));
    }
    return STOKESMG_OK;
}

int stokes_apply(stokesmg_t* h, int level, int dtype, const void* x, void* y, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_level_dtype(h, level, dtype)) return rc;
    if (!x || !y) return h->fail(STOKESMG_EINVAL, "null vector");
    const size_t es = dtype == STOKESMG_F64 ? 8 : 4;
    if (overlap(x, y, size_t(level_total(h, level)) * es)) return h->fail(STOKESMG_EINVAL, "x and y overlap");
    const bool f64 = dtype == STOKESMG_F64;
    const void* tab = h->ws + (f64 ? h->tab_f64[level] : h->tab_f32[level]);
    SMG_HIP(h, smg::launch_apply(h->cfg.k, f64, false, x, nullptr, y, tab, h->lv[level].n,
                                 static_cast<hipStream_t>(stream)));
    return STOKESMG_OK;
}

int stokes_residual(stokesmg_t* h, int level, int dtype, const void* b, const void* x, void* r, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_level_dtype(h, level, dtype)) return rc;
    if (!x || !b || !r) return h->fail(STOKESMG_EINVAL, "null vector");
    const size_t es = dtype == STOKESMG_F64 ? 8 : 4;
    const size_t bytes = size_t(level_total(h, level)) * es;
    if (overlap(x, r, bytes) || overlap(b, r, bytes)) return h->fail(STOKESMG_EINVAL, "r overlaps x or b");
    const bool f64 = dtype == STOKESMG_F64;
    const void* tab = h->ws + (f64 ? h->tab_f64[level] : h->tab_f32[level]);
    SMG_HIP(h, smg::launch_apply(h->cfg.k, f64, true, x, b, r, tab, h->lv[level].n,
                                 static_cast<hipStream_t>(stream)));
    return STOKESMG_OK;
}

}  // extern "C"
