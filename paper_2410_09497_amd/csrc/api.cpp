// C ABI of libstokesmg (include/stokesmg.h): handle, workspace, operator.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "apply.hpp"
#include "handle.hpp"
#include "mlp.hpp"
#include "patch.hpp"
#include "patch_tables.hpp"
#include "stencil_tables.hpp"

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

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
    // the kernels carry the method's penalty gamma = 2 (k+1)^2 / h as compile-time constants
    if (cfg->penalty_factor != 2.0) return STOKESMG_EUNSUPPORTED;
    if (!(cfg->cg_rtol >= 0) || cfg->cg_max_it < 0) return STOKESMG_EINVAL;
    stokesmg* h = new (std::nothrow) stokesmg;
    if (!h) return STOKESMG_ENOMEM;
    h->cfg = *cfg;
    h->n_levels = L;
    try {
        smg::Ref1D ref(k);
        for (int l = 0; l < L; ++l) {
            const int nl = n >> (L - 1 - l);
            h->lv.push_back(smg::build_level_tables(ref, nl, cfg->penalty_factor));
            h->lv.back().patch = smg::build_patch_tables(ref, nl, cfg->penalty_factor);
        }
        h->tr.resize(L);
        for (int l = 1; l < L; ++l) h->tr[l] = smg::build_transfer(ref, n >> (L - l));
        const int n0 = n >> (L - 1);
        const int64_t N0 = level_total(h, 0);
        if (N0 <= 1000) h->coarse_pinv = smg::coarse_pseudo_inverse(ref, n0, cfg->penalty_factor, &h->N0);
    } catch (const std::exception& e) {
        delete h;
        return STOKESMG_EINVAL;
    }
    size_t off = 0;
    const size_t tsz = smg::tab_size(k), psz = smg::patch_tab_size(k);
    for (int l = 0; l < L; ++l) {
        h->tab_f64.push_back(off);
        off = align256(off + tsz * sizeof(double));
        h->tab_f32.push_back(off);
        off = align256(off + tsz * sizeof(float));
        h->ptab_f64.push_back(off);
        off = align256(off + psz * sizeof(double));
        h->ptab_f32.push_back(off);
        off = align256(off + psz * sizeof(float));
    }
    h->cg_counter = off;
    off = align256(off + 2 * sizeof(unsigned long long));
    h->r_vec = off;
    off = align256(off + size_t(level_total(h, L - 1)) * sizeof(double));
    h->c_vec = off;
    off = align256(off + size_t(level_total(h, L - 1)) * sizeof(double));
    h->tro.resize(L);
    for (int l = 1; l < L; ++l) {
        auto& T = h->tr[l];
        auto& o = h->tro[l];
        auto put = [&](const smg::Rows1D& R, size_t& oi, size_t& ow, int& w) {
            oi = off;
            off = align256(off + R.idx.size() * sizeof(int));
            ow = off;
            off = align256(off + R.w.size() * sizeof(double));
            w = R.width;
        };
        put(T.pd, o.pd_i, o.pd_w, o.wpd);
        put(T.pc, o.pc_i, o.pc_w, o.wpc);
        put(T.rd, o.rd_i, o.rd_w, o.wrd);
        put(T.rc, o.rc_i, o.rc_w, o.wrc);
    }
    h->coarse_off = off;
    off = align256(off + h->coarse_pinv.size() * sizeof(double));
    for (int l = 0; l + 1 < L; ++l) {
        h->xl.push_back(off);
        off = align256(off + size_t(level_total(h, l)) * sizeof(double));
        h->bl.push_back(off);
        off = align256(off + size_t(level_total(h, l)) * sizeof(double));
    }
    h->wg_off = off;
    off = align256(off + (k + 1) * sizeof(double));
    h->scratch_off = off;
    off = align256(off + size_t(stokesmg::kScratch) * sizeof(double));
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
    auto upload = [&](const std::vector<double>& t, size_t o64, size_t o32) -> int {
        if (t.empty()) return STOKESMG_OK;
        std::vector<float> tf(t.begin(), t.end());
        SMG_HIP(h, hipMemcpyAsync(h->ws + o64, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, st));
        SMG_HIP(h, hipMemcpyAsync(h->ws + o32, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice, st));
        // the host buffers die at scope exit: finish the copies first
        SMG_HIP(h, hipStreamSynchronize(st));
        return STOKESMG_OK;
    };
    for (int l = 0; l < h->n_levels; ++l) {
        if (int rc = upload(h->lv[l].stencil, h->tab_f64[l], h->tab_f32[l])) return rc;
        if (int rc = upload(h->lv[l].patch, h->ptab_f64[l], h->ptab_f32[l])) return rc;
    }
    for (int l = 1; l < h->n_levels; ++l) {
        const auto& T = h->tr[l];
        const auto& o = h->tro[l];
        const smg::Rows1D* R[4] = {&T.pd, &T.pc, &T.rd, &T.rc};
        const size_t oi[4] = {o.pd_i, o.pc_i, o.rd_i, o.rc_i}, ow[4] = {o.pd_w, o.pc_w, o.rd_w, o.rc_w};
        for (int q = 0; q < 4; ++q) {
            SMG_HIP(h, hipMemcpyAsync(h->ws + oi[q], R[q]->idx.data(), R[q]->idx.size() * sizeof(int),
                                      hipMemcpyHostToDevice, st));
            SMG_HIP(h, hipMemcpyAsync(h->ws + ow[q], R[q]->w.data(), R[q]->w.size() * sizeof(double),
                                      hipMemcpyHostToDevice, st));
        }
    }
    if (!h->coarse_pinv.empty())
        SMG_HIP(h, hipMemcpyAsync(h->ws + h->coarse_off, h->coarse_pinv.data(), h->coarse_pinv.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st));
    {
        smg::Ref1D ref(h->cfg.k);
        SMG_HIP(h, hipMemcpyAsync(h->ws + h->wg_off, ref.wg.data(), ref.wg.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st));
        SMG_HIP(h, hipStreamSynchronize(st));
    }
    SMG_HIP(h, hipMemsetAsync(h->ws + h->cg_counter, 0, 2 * sizeof(unsigned long long), st));
    SMG_HIP(h, hipStreamSynchronize(st));
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

int patch_smooth(stokesmg_t* h, int level, int dtype, void* x, const void* b, int n_sweeps, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_level_dtype(h, level, dtype)) return rc;
    if (!x || !b || n_sweeps < 0) return h->fail(STOKESMG_EINVAL, "null vector or negative sweep count");
    if (h->lv[level].n < 2) return h->fail(STOKESMG_EINVAL, "level has no interior vertex (n < 2)");
    const size_t es = dtype == STOKESMG_F64 ? 8 : 4;
    const size_t bytes = size_t(level_total(h, level)) * es;
    if (overlap(x, b, bytes) || ranges_overlap(x, bytes, h->ws, h->ws_bytes) ||
        ranges_overlap(b, bytes, h->ws, h->ws_bytes))
        return h->fail(STOKESMG_EINVAL, "x, b and the workspace must not overlap");
    const bool f64 = dtype == STOKESMG_F64;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int s = 0; s < n_sweeps; ++s)
        if (int rc = smg::smooth_sweep(h, level, f64, x, b, st, nullptr)) return rc;
    return STOKESMG_OK;
}

int stokesmg_cg_stats(stokesmg_t* h, int64_t* iterations, int64_t* solves, int reset, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (!h->ws) return h->fail(STOKESMG_ENOMEM, "no workspace set");
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long c[2] = {0, 0};
    SMG_HIP(h, hipMemcpyAsync(c, h->ws + h->cg_counter, sizeof(c), hipMemcpyDeviceToHost, st));
    SMG_HIP(h, hipStreamSynchronize(st));
    if (iterations) *iterations = int64_t(c[0]);
    if (solves) *solves = int64_t(c[1]);
    if (reset) {
        SMG_HIP(h, hipMemsetAsync(h->ws + h->cg_counter, 0, 2 * sizeof(unsigned long long), st));
        SMG_HIP(h, hipStreamSynchronize(st));
    }
    return STOKESMG_OK;
}

}  // extern "C"
