// Learned local solver: host orchestration of the MLP kernels (forward,
// backward, Adam, training loop), its use inside the smoother, and the
// capture of training pairs from exact local solves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "apply.hpp"
#include "handle.hpp"
#include "mg_kernels.hpp"
#include "mlp.hpp"
#include "mlp_kernels.hpp"
#include "patch.hpp"
#include "direct.hpp"

namespace {

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

int patch_dim(int k) { return 3 * (2 * k + 1) * (2 * k + 2) * (2 * k + 2) + (2 * k + 2) * (2 * k + 2) * (2 * k + 2); }

int64_t param_count(int d, int H) { return int64_t(d) * H + H + int64_t(H) * H + H + int64_t(H) * d + d; }

// lays the MLP workspace out for max_rows rows; returns its size in bytes
size_t layout(stokesmg::Mlp& m, int d, int H, int64_t R) {
    m.d = d;
    m.H = H;
    m.P = param_count(d, H);
    m.rows = R;
    size_t off = 0;
    auto put = [&](size_t& o, size_t bytes) {
        o = off;
        off = a256(off + bytes);
    };
    const size_t f = sizeof(float);
    put(m.params, m.P * f);
    put(m.grads, m.P * f);
    put(m.m, m.P * f);
    put(m.v, m.P * f);
    put(m.Z1, R * H * f);
    put(m.H1, R * H * f);
    put(m.Z2, R * H * f);
    put(m.H2, R * H * f);
    put(m.Y, R * d * f);
    put(m.dY, R * d * f);
    put(m.dZ2, R * H * f);
    put(m.dZ1, R * H * f);
    put(m.X, R * d * f);
    put(m.s, R * f);
    m.split_floats = size_t(16) * d * H;
    put(m.split, m.split_floats * f);
    put(m.lossp, smg::kLossBlocks * sizeof(double));
    put(m.loss, f);
    put(m.colp, size_t(smg::kColsumSplit) * (d > H ? d : H) * f);
    put(m.brows, R * sizeof(int));
    put(m.acc, sizeof(double));
    // the Direct solver's matrices, one per patch type, FP32 then BF16 (degrees 1..3 only)
    int dk = 0, dn = 0;
    smg::direct_dims(d, &dk, &dn);
    put(m.direct, d <= patch_dim(3) ? size_t(smg::kDirectTypes) * dn * dk * (f + 2) : 0);
    return off;
}

template <typename T>
T* at(const stokesmg* h, size_t off) {
    return reinterpret_cast<T*>(h->mlp.ws + off);
}

// parameter sub-arrays inside a parameter-shaped vector
struct Parts {
    float *W1, *b1, *W2, *b2, *W3, *b3;
};
Parts parts(float* base, int d, int H) {
    Parts p;
    p.W1 = base;
    p.b1 = p.W1 + size_t(d) * H;
    p.W2 = p.b1 + H;
    p.b2 = p.W2 + size_t(H) * H;
    p.W3 = p.b2 + H;
    p.b3 = p.W3 + size_t(H) * d;
    return p;
}

// Y = net(X) for n <= rows rows; rows of X through xrows if given; keeps
// the pre-activations Z1, Z2 when `keep`.
int forward(stokesmg* h, bool bf16, const float* X, const int* xrows, int n, float* Y, bool keep, hipStream_t st) {
    auto& m = h->mlp;
    const int d = m.d, H = m.H;
    Parts w = parts(at<float>(h, m.params), d, H);
    float *Z1 = at<float>(h, m.Z1), *H1 = at<float>(h, m.H1), *Z2 = at<float>(h, m.Z2), *H2 = at<float>(h, m.H2);
    using smg::Epi;
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::BiasGelu, false, false, n, H, d, X, d, xrows, w.W1, H, H1, H, w.b1,
                                keep ? Z1 : nullptr, H, nullptr, 0, st));
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::BiasGelu, false, false, n, H, H, H1, H, nullptr, w.W2, H, H2, H, w.b2,
                                keep ? Z2 : nullptr, H, nullptr, 0, st));
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::Bias, false, false, n, d, H, H2, H, nullptr, w.W3, d, Y, d, w.b3, nullptr,
                                0, nullptr, 0, st));
    return STOKESMG_OK;
}

// gradients of mean((net(X) - T)^2) into g (parameter-shaped), loss into *loss
int backward(stokesmg* h, bool bf16, const float* X, const int* xrows, const float* T, int n, float* g, float* loss,
             hipStream_t st) {
    auto& m = h->mlp;
    const int d = m.d, H = m.H;
    if (int rc = forward(h, bf16, X, xrows, n, at<float>(h, m.Y), true, st)) return rc;
    Parts w = parts(at<float>(h, m.params), d, H);
    Parts gp = parts(g, d, H);
    float *Z1 = at<float>(h, m.Z1), *H1 = at<float>(h, m.H1), *Z2 = at<float>(h, m.Z2), *H2 = at<float>(h, m.H2);
    float *Y = at<float>(h, m.Y), *dY = at<float>(h, m.dY), *dZ2 = at<float>(h, m.dZ2), *dZ1 = at<float>(h, m.dZ1);
    float* split = at<float>(h, m.split);
    float* colp = at<float>(h, m.colp);
    using smg::Epi;
    SMG_HIP(h, smg::launch_mse_grad(Y, T, xrows, n, d, dY, at<double>(h, m.lossp), loss, st));
    // output layer: dW3 = H2^T dY, db3 = colsum dY
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::Store, true, false, H, d, n, H2, H, nullptr, dY, d, gp.W3, d, nullptr,
                                nullptr, 0, split, m.split_floats, st));
    SMG_HIP(h, smg::launch_colsum(dY, d, n, d, colp, gp.b3, st));
    // dZ2 = (dY W3^T) * gelu'(Z2)
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::GeluGrad, false, true, n, H, d, dY, d, nullptr, w.W3, d, dZ2, H, nullptr,
                                Z2, H, nullptr, 0, st));
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::Store, true, false, H, H, n, H1, H, nullptr, dZ2, H, gp.W2, H, nullptr,
                                nullptr, 0, split, m.split_floats, st));
    SMG_HIP(h, smg::launch_colsum(dZ2, H, n, H, colp, gp.b2, st));
    // dZ1 = (dZ2 W2^T) * gelu'(Z1)
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::GeluGrad, false, true, n, H, H, dZ2, H, nullptr, w.W2, H, dZ1, H, nullptr,
                                Z1, H, nullptr, 0, st));
    // dW1 = X^T dZ1 (rows of X through xrows)
    SMG_HIP(h, smg::launch_gemm(bf16, Epi::Store, true, false, d, H, n, X, d, xrows, dZ1, H, gp.W1, H, nullptr,
                                nullptr, 0, split, m.split_floats, st));
    SMG_HIP(h, smg::launch_colsum(dZ1, H, n, H, colp, gp.b1, st));
    return STOKESMG_OK;
}

int adam(stokesmg* h, const float* g, float lr, hipStream_t st) {
    auto& m = h->mlp;
    m.step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = float(1.0 - std::pow(b1, double(m.step))), c2 = float(1.0 - std::pow(b2, double(m.step)));
    SMG_HIP(h, smg::launch_adam(at<float>(h, m.params), g, at<float>(h, m.m), at<float>(h, m.v), size_t(m.P), lr,
                                float(b1), float(b2), 1e-8f, c1, c2, st));
    return STOKESMG_OK;
}

int check_mlp(stokesmg* h, bool need_params) {
    if (!h->mlp.ws) return h->fail(STOKESMG_ENOMEM, "no MLP workspace set");
    if (need_params && !h->mlp.ready) return h->fail(STOKESMG_EINVAL, "MLP parameters not initialized");
    return STOKESMG_OK;
}

int check_mode(stokesmg* h, int mode) {
    if (mode != STOKESMG_MLP_BF16 && mode != STOKESMG_MLP_F32) return h->fail(STOKESMG_EINVAL, "bad MLP mode");
    return STOKESMG_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

uint64_t splitmix64(uint64_t& state) {
    // SplitMix64 (Steele, Lea & Flood 2014)
    uint64_t z = (state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

}  // namespace

namespace smg {

int mlp_interior_solve(stokesmg* h, int level, bool f64, void* x, const void* r, int colour, hipStream_t st) {
    auto& m = h->mlp;
    const int n = h->lv[level].n, k = h->cfg.k;
    const int64_t np = interior_count(n, colour);
    const bool bf16 = h->mlp_mode == STOKESMG_MLP_BF16;
    float *X = at<float>(h, m.X), *Y = at<float>(h, m.Y), *s = at<float>(h, m.s);
    for (int64_t p0 = 0; p0 < np; p0 += m.rows) {
        const int cnt = int(std::min<int64_t>(m.rows, np - p0));
        SMG_HIP(h, launch_patch_gather(f64, r, n, k, colour, int(p0), cnt, X, m.d, s, st));
        if (int rc = forward(h, bf16, X, nullptr, cnt, Y, false, st)) return rc;
        SMG_HIP(h, launch_patch_scatter(f64, x, n, k, colour, int(p0), cnt, Y, m.d, s, h->mlp_omega, st));
    }
    return STOKESMG_OK;
}

// every patch of one colour by the Direct solver: one launch that gathers
// each patch's residual, multiplies it by its patch type's normalized map on
// the matrix cores (BF16 or FP32 operands per the MLP mode, FP32
// accumulation) and adds the correction
int direct_solve(stokesmg* h, int level, bool f64, void* x, const void* r, int colour, hipStream_t st) {
    const int n = h->lv[level].n, k = h->cfg.k;
    const bool bf16 = h->mlp_mode == STOKESMG_MLP_BF16;
    int dk = 0, dn = 0;
    direct_dims(h->mlp.d, &dk, &dn);
    const size_t f32_bytes = size_t(kDirectTypes) * dn * dk * sizeof(float);
    const void* Bt = h->mlp.ws + h->mlp.direct + (bf16 ? f32_bytes : 0);
    SMG_HIP(h, launch_direct_patch(f64, bf16, r, x, n, k, colour_groups(n, colour, true), Bt, st));
    return STOKESMG_OK;
}

// interior patches of one colour with the Schur CG started from the network's pressure
int mlp_warm_solve(stokesmg* h, int level, bool f64, void* x, const void* r, const void* ptab, int colour,
                   unsigned long long* counters, hipStream_t st) {
    auto& m = h->mlp;
    const int n = h->lv[level].n, k = h->cfg.k;
    const int64_t np = interior_count(n, colour);
    const bool bf16 = h->mlp_mode == STOKESMG_MLP_BF16;
    float *X = at<float>(h, m.X), *Y = at<float>(h, m.Y), *s = at<float>(h, m.s);
    for (int64_t p0 = 0; p0 < np; p0 += m.rows) {
        const int cnt = int(std::min<int64_t>(m.rows, np - p0));
        SMG_HIP(h, launch_patch_gather(f64, r, n, k, colour, int(p0), cnt, X, m.d, s, st));
        if (int rc = forward(h, bf16, X, nullptr, cnt, Y, false, st)) return rc;
        SMG_HIP(h, launch_patch_solve_warm(k, f64, x, r, ptab, n, colour, h->cfg.cg_rtol, h->cfg.cg_max_it, counters,
                                           int(p0), cnt, Y, m.d, s, st));
    }
    return STOKESMG_OK;
}

int smooth_sweep(stokesmg* h, int level, bool f64, void* x, const void* b, hipStream_t st, const Capture* cap,
                 void* r_in, unsigned long long* counters_in, bool own_counters) {
    const int n = h->lv[level].n, k = h->cfg.k;
    const void* tab = h->ws + (f64 ? h->tab_f64[level] : h->tab_f32[level]);
    const void* ptab = h->ws + (f64 ? h->ptab_f64[level] : h->ptab_f32[level]);
    void* r = r_in ? r_in : h->ws + h->r_vec;
    unsigned long long* counters = own_counters ? counters_in : reinterpret_cast<unsigned long long*>(h->ws + h->cg_counter);
    const bool learned = h->local_solver == STOKESMG_LOCAL_MLP && !cap;
    const bool warm = h->local_solver == STOKESMG_LOCAL_MLP_WARM && !cap;
    const bool direct = h->local_solver == STOKESMG_LOCAL_DIRECT && !cap;
    const bool exact_mf = h->local_solver == STOKESMG_LOCAL_EXACT_BF16 && !cap;
    if (direct && !h->mlp.direct_ready)
        return h->fail(STOKESMG_EINVAL, "the Direct solver needs stokesmg_direct_setup() after mlp_set_workspace()");
    if (exact_mf && f64)
        return h->fail(STOKESMG_EINVAL, "the BF16 eigenbasis products run in an FP32 cycle (dtype F32)");
    const size_t N = size_t(level_total(h, level));
    for (int c = 0; c < 8; ++c) {
        SMG_HIP(h, launch_apply(k, f64, true, x, b, r, tab, n, st));
        if (cap) {
            // exact correction into c_vec, pairs of the interior patches, then x += c_vec
            auto& m = h->mlp;
            void* cv = h->ws + h->c_vec;
            const int64_t np = interior_count(n, c);
            const int64_t room = std::max<int64_t>(0, std::min<int64_t>(np, cap->cap - *cap->n));
            float* s = at<float>(h, m.s);
            SMG_HIP(h, launch_zero(f64, cv, N, st));
            SMG_HIP(h, launch_patch_solve(k, f64, cv, r, ptab, n, c, h->cfg.cg_rtol, h->cfg.cg_max_it, counters,
                                          false, st));
            for (int64_t p0 = 0; p0 < room; p0 += m.rows) {
                const int cnt = int(std::min<int64_t>(m.rows, room - p0));
                float* Xr = cap->X + size_t(*cap->n + p0) * m.d;
                float* Tr = cap->T + size_t(*cap->n + p0) * m.d;
                SMG_HIP(h, launch_patch_gather(f64, r, n, k, c, int(p0), cnt, Xr, m.d, s, st));
                SMG_HIP(h, launch_patch_gather_diff(f64, cv, nullptr, n, k, c, int(p0), cnt, Tr, m.d, s, st));
            }
            *cap->n += room;
            SMG_HIP(h, launch_add(f64, x, cv, N, st));
        } else if (learned && interior_count(n, c) > 0) {
            SMG_HIP(h, launch_patch_solve(k, f64, x, r, ptab, n, c, h->cfg.cg_rtol, h->cfg.cg_max_it, counters,
                                          true, st));
            if (int rc = mlp_interior_solve(h, level, f64, x, r, c, st)) return rc;
        } else if (direct) {
            if (int rc = direct_solve(h, level, f64, x, r, c, st)) return rc;
        } else if (exact_mf) {
            SMG_HIP(h, launch_patch_solve_mf(k, x, r, ptab, n, c, h->cfg.cg_rtol, h->cfg.cg_max_it, counters, st));
        } else if (warm && interior_count(n, c) > 0) {
            SMG_HIP(h, launch_patch_solve(k, f64, x, r, ptab, n, c, h->cfg.cg_rtol, h->cfg.cg_max_it, counters,
                                          true, st));
            if (int rc = mlp_warm_solve(h, level, f64, x, r, ptab, c, counters, st)) return rc;
        } else {
            SMG_HIP(h, launch_patch_solve(k, f64, x, r, ptab, n, c, h->cfg.cg_rtol, h->cfg.cg_max_it, counters,
                                          false, st));
        }
    }
    return STOKESMG_OK;
}

}  // namespace smg

extern "C" {

int mlp_dims(const stokesmg_t* h, int64_t* d, int64_t* n_params) {
    if (!h) return STOKESMG_EINVAL;
    const int dd = patch_dim(h->cfg.k);
    if (d) *d = dd;
    if (n_params) *n_params = param_count(dd, STOKESMG_MLP_HIDDEN);
    return STOKESMG_OK;
}

int mlp_workspace_size(const stokesmg_t* h, int64_t max_rows, size_t* bytes) {
    if (!h || !bytes || max_rows < 1 || max_rows > (int64_t(1) << 24)) return STOKESMG_EINVAL;
    stokesmg::Mlp m;
    *bytes = layout(m, patch_dim(h->cfg.k), STOKESMG_MLP_HIDDEN, max_rows);
    return STOKESMG_OK;
}

int mlp_set_workspace(stokesmg_t* h, void* dev_ptr, size_t bytes, int64_t max_rows) {
    if (!h) return STOKESMG_EINVAL;
    if (max_rows < 1 || max_rows > (int64_t(1) << 24)) return h->fail(STOKESMG_EINVAL, "max_rows out of range");
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0)
        return h->fail(STOKESMG_EINVAL, "MLP workspace must be a non-null, 256-byte aligned device pointer");
    stokesmg::Mlp m;
    const size_t need = layout(m, patch_dim(h->cfg.k), STOKESMG_MLP_HIDDEN, max_rows);
    if (bytes < need) return h->fail(STOKESMG_ENOMEM, "MLP workspace smaller than mlp_workspace_size()");
    if (h->ws && ranges_overlap(dev_ptr, bytes, h->ws, h->ws_bytes))
        return h->fail(STOKESMG_EINVAL, "MLP workspace overlaps the main workspace");
    m.ws = static_cast<char*>(dev_ptr);
    m.bytes = bytes;
    h->mlp = m;
    return STOKESMG_OK;
}

int mlp_init(stokesmg_t* h, uint64_t seed, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, false)) return rc;
    auto& m = h->mlp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<float> p(size_t(m.P), 0.0f);
    uint64_t state = seed;
    const int d = m.d, H = m.H;
    auto fill = [&](size_t off, size_t count, int fan_in) {
        const double a = std::sqrt(3.0 / fan_in);
        for (size_t i = 0; i < count; ++i) {
            const double u = double(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0);
            p[off + i] = float((2.0 * u - 1.0) * a);
        }
    };
    const size_t oW1 = 0, oW2 = size_t(d) * H + H, oW3 = oW2 + size_t(H) * H + H;
    fill(oW1, size_t(d) * H, d);
    fill(oW2, size_t(H) * H, H);
    fill(oW3, size_t(H) * d, H);
    SMG_HIP(h, hipMemcpyAsync(m.ws + m.params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, st));
    SMG_HIP(h, smg::launch_zero(false, m.ws + m.m, size_t(m.P), st));
    SMG_HIP(h, smg::launch_zero(false, m.ws + m.v, size_t(m.P), st));
    SMG_HIP(h, hipStreamSynchronize(st));
    m.step = 0;
    m.ready = true;
    return STOKESMG_OK;
}

int mlp_get_state(stokesmg_t* h, float* state, int64_t* step, void* stream) {
    if (!h || !state) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, true)) return rc;
    auto& m = h->mlp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t b = size_t(m.P) * sizeof(float);
    SMG_HIP(h, hipMemcpyAsync(state, m.ws + m.params, b, hipMemcpyDeviceToDevice, st));
    SMG_HIP(h, hipMemcpyAsync(state + m.P, m.ws + m.m, b, hipMemcpyDeviceToDevice, st));
    SMG_HIP(h, hipMemcpyAsync(state + 2 * m.P, m.ws + m.v, b, hipMemcpyDeviceToDevice, st));
    if (step) *step = m.step;
    return STOKESMG_OK;
}

int mlp_set_state(stokesmg_t* h, const float* state, int64_t step, void* stream) {
    if (!h || !state || step < 0) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, false)) return rc;
    auto& m = h->mlp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t b = size_t(m.P) * sizeof(float);
    SMG_HIP(h, hipMemcpyAsync(m.ws + m.params, state, b, hipMemcpyDeviceToDevice, st));
    SMG_HIP(h, hipMemcpyAsync(m.ws + m.m, state + m.P, b, hipMemcpyDeviceToDevice, st));
    SMG_HIP(h, hipMemcpyAsync(m.ws + m.v, state + 2 * m.P, b, hipMemcpyDeviceToDevice, st));
    m.step = step;
    m.ready = true;
    return STOKESMG_OK;
}

int mlp_forward(stokesmg_t* h, int mode, const float* X, float* Y, int64_t n, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, true)) return rc;
    if (int rc = check_mode(h, mode)) return rc;
    if (n < 0 || (n > 0 && (!X || !Y))) return h->fail(STOKESMG_EINVAL, "bad rows or null pointer");
    if (!aligned16(X) || !aligned16(Y)) return h->fail(STOKESMG_EINVAL, "X and Y must be 16-byte aligned");
    auto& m = h->mlp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int64_t r0 = 0; r0 < n; r0 += m.rows) {
        const int cnt = int(std::min<int64_t>(m.rows, n - r0));
        if (int rc = forward(h, mode == STOKESMG_MLP_BF16, X + size_t(r0) * m.d, nullptr, cnt, Y + size_t(r0) * m.d,
                             false, st))
            return rc;
    }
    return STOKESMG_OK;
}

int mlp_backward(stokesmg_t* h, int mode, const float* X, const float* T, int64_t n, float* grads, float* loss,
                 void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, true)) return rc;
    if (int rc = check_mode(h, mode)) return rc;
    if (!X || !T || !grads || !loss) return h->fail(STOKESMG_EINVAL, "null pointer");
    if (n < 1 || n > h->mlp.rows) return h->fail(STOKESMG_EINVAL, "n must be in 1..max_rows");
    if (!aligned16(X) || !aligned16(T) || !aligned16(grads))
        return h->fail(STOKESMG_EINVAL, "X, T and grads must be 16-byte aligned");
    return backward(h, mode == STOKESMG_MLP_BF16, X, nullptr, T, int(n), grads, loss,
                    static_cast<hipStream_t>(stream));
}

int mlp_adam_step(stokesmg_t* h, const float* grads, float lr, void* stream) {
    if (!h || !grads) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, true)) return rc;
    return adam(h, grads, lr, static_cast<hipStream_t>(stream));
}

int mlp_train(stokesmg_t* h, int mode, const float* X, const float* T, int64_t n, int epochs, int batch, float lr,
              uint64_t seed, float* loss_hist, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, true)) return rc;
    if (int rc = check_mode(h, mode)) return rc;
    auto& m = h->mlp;
    if (!X || !T || n < 1 || n >= (int64_t(1) << 31) || epochs < 0 || batch < 1 || batch > m.rows)
        return h->fail(STOKESMG_EINVAL, "bad training arguments");
    if (!aligned16(X) || !aligned16(T)) return h->fail(STOKESMG_EINVAL, "X and T must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool bf16 = mode == STOKESMG_MLP_BF16;
    const int64_t spe = (n + batch - 1) / batch;
    const double total = double(spe) * epochs;
    int* rows = at<int>(h, m.brows);
    double* acc = at<double>(h, m.acc);
    float* g = at<float>(h, m.grads);
    float* loss = at<float>(h, m.loss);
    int64_t t = 0;
    for (int e = 0; e < epochs; ++e) {
        uint64_t ks = seed ^ (0xd1b54a32d192ed03ULL * uint64_t(e + 1));
        const uint64_t key = splitmix64(ks);
        SMG_HIP(h, smg::launch_zero(true, acc, 1, st));
        for (int64_t b = 0; b < spe; ++b, ++t) {
            const int64_t start = b * batch;
            const int cnt = int(std::min<int64_t>(batch, n - start));
            SMG_HIP(h, smg::launch_batch_rows(rows, start, cnt, n, key, st));
            if (int rc = backward(h, bf16, X, rows, T, cnt, g, loss, st)) return rc;
            SMG_HIP(h, smg::launch_accumulate(loss, acc, st));
            const float lr_t = float(0.5 * lr * (1.0 + std::cos(M_PI * double(t) / total)));
            if (int rc = adam(h, g, lr_t, st)) return rc;
        }
        double sum = 0.0;
        SMG_HIP(h, hipMemcpyAsync(&sum, acc, sizeof(double), hipMemcpyDeviceToHost, st));
        SMG_HIP(h, hipStreamSynchronize(st));
        if (loss_hist) loss_hist[e] = float(sum / double(spe));
    }
    return STOKESMG_OK;
}

int mlp_collect_pairs(stokesmg_t* h, const double* b, double* x, float* X, float* T, int64_t cap, int64_t* n,
                      void* stream) {
    if (!h || !n) return STOKESMG_EINVAL;
    if (int rc = check_mlp(h, false)) return rc;
    if (!b || !x || (cap > 0 && (!X || !T)) || *n < 0 || cap < 0)
        return h->fail(STOKESMG_EINVAL, "bad pair-capture arguments");
    smg::Capture c{X, T, cap, n};
    return smg::vcycle_run(h, true, b, x, static_cast<hipStream_t>(stream), &c);
}

int stokesmg_set_local_solver(stokesmg_t* h, int local_solver, int mlp_mode, double mlp_damping) {
    if (!h) return STOKESMG_EINVAL;
    if (!(mlp_damping > 0.0 && mlp_damping <= 1.0)) return h->fail(STOKESMG_EINVAL, "mlp_damping must be in (0, 1]");
    if (local_solver != STOKESMG_LOCAL_EXACT && local_solver != STOKESMG_LOCAL_MLP &&
        local_solver != STOKESMG_LOCAL_MLP_WARM && local_solver != STOKESMG_LOCAL_DIRECT &&
        local_solver != STOKESMG_LOCAL_EXACT_BF16)
        return h->fail(STOKESMG_EINVAL, "unknown local solver");
    if (local_solver == STOKESMG_LOCAL_EXACT_BF16 && h->cfg.k > 3)
        return h->fail(STOKESMG_EUNSUPPORTED, "the BF16 eigenbasis products are built for degrees 1..3");
    if (int rc = check_mode(h, mlp_mode)) return rc;
    if (local_solver == STOKESMG_LOCAL_DIRECT) {
        if (!h->mlp.ws || !h->mlp.direct_ready)
            return h->fail(STOKESMG_EINVAL, "the Direct solver needs stokesmg_direct_setup() first");
    } else if (local_solver == STOKESMG_LOCAL_MLP || local_solver == STOKESMG_LOCAL_MLP_WARM) {
        if (int rc = check_mlp(h, true)) return rc;
    }
    h->local_solver = local_solver;
    h->mlp_mode = mlp_mode;
    h->mlp_omega = mlp_damping;
    return STOKESMG_OK;
}

int stokesmg_direct_matrix(const stokesmg_t* h, int type, double* M) {
    if (!h || !M || type < 0 || type >= smg::kDirectTypes) return STOKESMG_EINVAL;
    if (h->cfg.k > 3) return STOKESMG_EUNSUPPORTED;
    try {
        const std::vector<double> D = smg::direct_type_map(smg::Ref1D(h->cfg.k), h->cfg.penalty_factor, type);
        std::memcpy(M, D.data(), D.size() * sizeof(double));
    } catch (const std::exception&) {
        return STOKESMG_EINVAL;
    }
    return STOKESMG_OK;
}

int stokesmg_direct_setup(stokesmg_t* h, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (h->cfg.k > 3) return h->fail(STOKESMG_EUNSUPPORTED, "the Direct solver is built for degrees 1..3");
    if (!h->mlp.ws) return h->fail(STOKESMG_ENOMEM, "no MLP workspace set (it holds the Direct solver's matrices)");
    std::vector<std::vector<double>> D;
    try {
        D = smg::direct_type_maps(smg::Ref1D(h->cfg.k), h->cfg.penalty_factor);
    } catch (const std::exception& e) {
        return h->fail(STOKESMG_EINVAL, e.what());
    }
    const int d = h->mlp.d;
    int dk = 0, dn = 0;
    smg::direct_dims(d, &dk, &dn);
    const size_t per = size_t(dn) * dk, total = smg::kDirectTypes * per;
    // per type M padded with zeros to dn x dk, [out][in]: FP32, then the same rounded to BF16 (nearest even)
    std::vector<float> Mf(total, 0.0f);
    std::vector<uint16_t> Mb(total, 0);
    for (int t = 0; t < smg::kDirectTypes; ++t)
        for (int o = 0; o < d; ++o)
            for (int i = 0; i < d; ++i) {
                const float v = float(D[t][size_t(o) * d + i]);
                uint32_t u;
                std::memcpy(&u, &v, 4);
                Mf[t * per + size_t(o) * dk + i] = v;
                Mb[t * per + size_t(o) * dk + i] = uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
            }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* dst = h->mlp.ws + h->mlp.direct;
    SMG_HIP(h, hipMemcpyAsync(dst, Mf.data(), total * sizeof(float), hipMemcpyHostToDevice, st));
    SMG_HIP(h, hipMemcpyAsync(dst + total * sizeof(float), Mb.data(), total * sizeof(uint16_t), hipMemcpyHostToDevice,
                              st));
    SMG_HIP(h, hipStreamSynchronize(st));
    h->mlp.direct_ready = true;
    return STOKESMG_OK;
}

int stokesmg_set_smoothing(stokesmg_t* h, int pre_sweeps, int post_sweeps) {
    if (!h) return STOKESMG_EINVAL;
    if (pre_sweeps < 0 || post_sweeps < 0 || pre_sweeps > 16 || post_sweeps > 16 || pre_sweeps + post_sweeps < 1)
        return h->fail(STOKESMG_EINVAL, "sweeps must be in 0..16, at least one in total");
    h->pre_sweeps = pre_sweeps;
    h->post_sweeps = post_sweeps;
    return STOKESMG_OK;
}

int stokesmg_set_fallback(stokesmg_t* h, double rho_ref) {
    if (!h) return STOKESMG_EINVAL;
    h->rho_ref = rho_ref;
    return STOKESMG_OK;
}

}  // extern "C"
