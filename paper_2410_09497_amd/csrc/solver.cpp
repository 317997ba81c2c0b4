// V-cycle (Sec. 3), FGMRES around it (Sec. 3.3) and the separable
// right-hand-side assembly of the manufactured problems.  Host orchestration;
// every vector operation is a device kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <vector>

#include "apply.hpp"
#include "handle.hpp"
#include "mg_kernels.hpp"
#include "mlp.hpp"
#include "patch.hpp"

namespace {

using smg::Rows1D;

int vcycle_level(stokesmg* h, int l, bool f64, const void* b, void* x, hipStream_t st, const smg::Capture* cap) {
    if (l == 0) {
        if (h->coarse_pinv.empty()) return h->fail(STOKESMG_EUNSUPPORTED, "coarsest level too large for the dense solve");
        SMG_HIP(h, smg::launch_coarse_gemv(f64, reinterpret_cast<const double*>(h->ws + h->coarse_off), b, x, h->N0, st));
        return STOKESMG_OK;
    }
    const int n = h->lv[l].n, k = h->cfg.k;
    const size_t N = size_t(level_total(h, l));
    const void* tab = h->ws + (f64 ? h->tab_f64[l] : h->tab_f32[l]);
    void* r = h->ws + h->r_vec;
    const smg::Capture* lc = (l == h->n_levels - 1) ? cap : nullptr;
    // pre-smoothing from x = 0
    SMG_HIP(h, smg::launch_zero(f64, x, N, st));
    for (int s = 0; s < h->pre_sweeps; ++s)
        if (int rc = smg::smooth_sweep(h, l, f64, x, b, st, lc)) return rc;
    // coarse-grid correction: b_{l-1} = P^T (b - K x), x += P P_{l-1}^{-1} b_{l-1}
    SMG_HIP(h, smg::launch_apply(k, f64, true, x, b, r, tab, n, st));
    const auto& o = h->tro[l];
    char* w = h->ws;
    void* bc = w + h->bl[l - 1];
    void* xc = w + h->xl[l - 1];
    const int N1f = h->lv[l].N1, N1c = h->lv[l - 1].N1;
    SMG_HIP(h, smg::launch_transfer(f64, false, r, bc, N1c, N1f, reinterpret_cast<const int*>(w + o.rd_i),
                                    reinterpret_cast<const double*>(w + o.rd_w), o.wrd,
                                    reinterpret_cast<const int*>(w + o.rc_i),
                                    reinterpret_cast<const double*>(w + o.rc_w), o.wrc, w + h->c_vec, st));
    if (int rc = vcycle_level(h, l - 1, f64, bc, xc, st, cap)) return rc;
    SMG_HIP(h, smg::launch_transfer(f64, true, xc, x, N1f, N1c, reinterpret_cast<const int*>(w + o.pd_i),
                                    reinterpret_cast<const double*>(w + o.pd_w), o.wpd,
                                    reinterpret_cast<const int*>(w + o.pc_i),
                                    reinterpret_cast<const double*>(w + o.pc_w), o.wpc, w + h->c_vec, st));
    // post-smoothing
    for (int s = 0; s < h->post_sweeps; ++s)
        if (int rc = smg::smooth_sweep(h, l, f64, x, b, st, lc)) return rc;
    return STOKESMG_OK;
}

int check_mg(stokesmg* h) {
    if (!h->ws) return h->fail(STOKESMG_ENOMEM, "no workspace set");
    for (int l = 1; l < h->n_levels; ++l)
        if (h->lv[l].n < 2) return h->fail(STOKESMG_EINVAL, "level without interior vertices");
    if (h->coarse_pinv.empty()) return h->fail(STOKESMG_EUNSUPPORTED, "coarsest level too large for the dense solve");
    return STOKESMG_OK;
}

// out[0..nv) = V_j . w on the host (one synchronization)
int host_dots(stokesmg* h, const double* V, size_t ld, const double* w, int nv, size_t n, double* out,
              hipStream_t st) {
    double* scr = reinterpret_cast<double*>(h->ws + h->scratch_off);
    const int nblocks = stokesmg::kPartialBlocks;
    double* partial = scr + stokesmg::kPartial;
    double* res = scr + stokesmg::kCoef;   // nv <= 61
    SMG_HIP(h, smg::launch_multidot(V, ld, w, nv, n, partial, nblocks, res, st));
    SMG_HIP(h, hipMemcpyAsync(out, res, nv * sizeof(double), hipMemcpyDeviceToHost, st));
    SMG_HIP(h, hipStreamSynchronize(st));
    return STOKESMG_OK;
}

// ------------------------------------------------ separable right-hand sides
// 1D factor functions of the manufactured problems
enum Fn { ONE, SINPI, COSPI };
double fn(int f, double x) {
    switch (f) {
        case SINPI: return std::sin(M_PI * x);
        case COSPI: return std::cos(M_PI * x);
        default: return 1.0;
    }
}
struct Term {       // coef * g0(x) g1(y) g2(z)
    double c;
    int g[3];
};

// 1D load vectors of function g against the basis of one direction kind on n cells:
// value[position] = int g phi_position (Gauss with k+2 points per cell), and the
// boundary vector bnd[position] = sum over the two ends s of g(s) (2 gamma phi(s) - n_s phi'(s))
void load_1d(const smg::Ref1D& r, int n, bool cont, const std::function<double(double)>& g, double gamma,
             std::vector<double>& val, std::vector<double>& bnd) {
    const int k = r.k, m = k + 1, N1 = n * m;
    const double h = 1.0 / n;
    std::vector<double> xq, wq;
    smg::gauss_rule(k + 2, xq, wq);
    if (!cont) {
        val.assign(N1, 0.0);
        bnd.assign(N1, 0.0);
        for (int c = 0; c < n; ++c)
            for (int a = 0; a < m; ++a) {
                double s = 0.0;
                for (size_t q = 0; q < xq.size(); ++q) s += wq[q] * h * g((c + xq[q]) * h) * smg::lagrange(r.xg, a, xq[q]);
                val[c * m + a] = s;
            }
        for (int a = 0; a < m; ++a) {
            bnd[a] += g(0.0) * (2.0 * gamma * r.eL[a] + r.dL[a] / h);                // n = -1: -n phi' = +phi'
            bnd[(n - 1) * m + a] += g(1.0) * (2.0 * gamma * r.eR[a] - r.dR[a] / h);
        }
    } else {
        std::vector<double> full(N1 + 1, 0.0), fb(N1 + 1, 0.0);
        for (int c = 0; c < n; ++c)
            for (int b = 0; b <= m; ++b) {
                double s = 0.0;
                for (size_t q = 0; q < xq.size(); ++q) s += wq[q] * h * g((c + xq[q]) * h) * smg::lagrange(r.xl, b, xq[q]);
                full[c * m + b] += s;
            }
        val.assign(full.begin() + 1, full.end() - 1);   // interior nodes only
        bnd.assign(N1 - 1, 0.0);   // the boundary nodes of the continuous basis are eliminated
    }
}

}  // namespace

namespace smg {

int vcycle_run(stokesmg* h, bool f64, const void* b, void* x, hipStream_t st, const Capture* cap) {
    if (int rc = check_mg(h)) return rc;
    return vcycle_level(h, h->n_levels - 1, f64, b, x, st, cap);
}

}  // namespace smg

extern "C" {

int vcycle(stokesmg_t* h, int dtype, const void* b, void* x, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (dtype != STOKESMG_F64 && dtype != STOKESMG_F32) return h->fail(STOKESMG_EINVAL, "dtype must be F64 or F32");
    if (int rc = check_mg(h)) return rc;
    if (!b || !x) return h->fail(STOKESMG_EINVAL, "null vector");
    const int L = h->n_levels - 1;
    const size_t bytes = size_t(level_total(h, L)) * (dtype == STOKESMG_F64 ? 8 : 4);
    if (ranges_overlap(b, bytes, x, bytes) || ranges_overlap(x, bytes, h->ws, h->ws_bytes) ||
        ranges_overlap(b, bytes, h->ws, h->ws_bytes))
        return h->fail(STOKESMG_EINVAL, "b, x and the workspace must not overlap");
    return vcycle_level(h, L, dtype == STOKESMG_F64, b, x, static_cast<hipStream_t>(stream), nullptr);
}

namespace {
// bytes of the solve workspace for FGMRES(m): V (m + 1 FP64 vectors), Z (m vectors in the V-cycle's
// precision: the FP32 cycle's output is kept as it is produced), w, and the V-cycle's input plus an
// FP64 copy of z_j (FP32 cycle) or its input and output (FP64 cycle)
size_t solve_ws_bytes(size_t N, int m, bool f32) {
    const size_t zs = f32 ? sizeof(float) : sizeof(double);
    const size_t extra = f32 ? N * sizeof(float) + N * sizeof(double) : 2 * N * sizeof(double);
    return size_t(m + 1) * N * sizeof(double) + size_t(m) * N * zs + N * sizeof(double) + extra + 256 + 3 * 256;
}
}  // namespace

int stokesmg_solve_workspace_size(const stokesmg_t* h, int restart, int vcycle_dtype, size_t* bytes) {
    if (!h || !bytes || restart < 1 || restart > 60) return STOKESMG_EINVAL;
    if (vcycle_dtype != STOKESMG_F64 && vcycle_dtype != STOKESMG_F32) return STOKESMG_EINVAL;
    *bytes = solve_ws_bytes(size_t(level_total(h, h->n_levels - 1)), restart, vcycle_dtype == STOKESMG_F32);
    return STOKESMG_OK;
}

int solve(stokesmg_t* h, const double* b, double* x, double rtol, int max_it, int restart_in, int vcycle_dtype,
          void* solve_ws, size_t solve_ws_bytes_in, stokesmg_info* info, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (int rc = check_mg(h)) return rc;
    if (!b || !x || !solve_ws || !(rtol > 0) || max_it < 1 || restart_in < 1 || restart_in > 60)
        return h->fail(STOKESMG_EINVAL, "bad solve arguments");
    if (vcycle_dtype != STOKESMG_F64 && vcycle_dtype != STOKESMG_F32)
        return h->fail(STOKESMG_EINVAL, "vcycle dtype must be F64 or F32");
    const bool f32 = vcycle_dtype == STOKESMG_F32;
    const int L = h->n_levels - 1;
    const size_t N = size_t(level_total(h, L));
    // the Krylov basis takes what the caller provided: restart is reduced to the largest length
    // whose vectors fit (a caller expecting a few steps sizes the workspace for a few vectors)
    int restart = restart_in;
    while (restart >= 1 && solve_ws_bytes(N, restart, f32) > solve_ws_bytes_in) --restart;
    if (restart < 1) return h->fail(STOKESMG_ENOMEM, "solve workspace too small for one Arnoldi step");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto t0 = std::chrono::steady_clock::now();
    const int k = h->cfg.k, n = h->lv[L].n;
    const size_t nb = N * sizeof(double);
    if (ranges_overlap(b, nb, x, nb) || ranges_overlap(x, nb, solve_ws, solve_ws_bytes_in) ||
        ranges_overlap(b, nb, solve_ws, solve_ws_bytes_in) || ranges_overlap(x, nb, h->ws, h->ws_bytes))
        return h->fail(STOKESMG_EINVAL, "b, x and the workspaces must not overlap");
    auto align = [](uintptr_t p) { return (p + 255) & ~uintptr_t(255); };
    double* base = reinterpret_cast<double*>(align(reinterpret_cast<uintptr_t>(solve_ws)));
    double* V = base;                              // restart + 1 FP64 vectors
    unsigned char* zb = reinterpret_cast<unsigned char*>(V + size_t(restart + 1) * N);
    const size_t zs = f32 ? sizeof(float) : sizeof(double);
    double* w = reinterpret_cast<double*>(align(reinterpret_cast<uintptr_t>(zb + size_t(restart) * N * zs)));
    // FP32 cycle: vin = FP32 input, z64 = FP64 copy of z_j; FP64 cycle: z_j is written in place, vin unused
    void* vin = w + N;
    double* z64 = reinterpret_cast<double*>(
        align(reinterpret_cast<uintptr_t>(static_cast<unsigned char*>(vin) + N * (f32 ? sizeof(float) : sizeof(double)))));
    auto zvec = [&](int j) -> void* { return zb + size_t(j) * N * zs; };
    const void* tab64 = h->ws + h->tab_f64[L];
    double* coef = reinterpret_cast<double*>(h->ws + h->scratch_off);   // device coefficients (<= 64)
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->fallback_iteration = -1;
    }
    // learned local solver: monitor the contraction and fall back to the exact solver for the rest
    // of the solve once it exceeds max(2 rho_ref, 1e-3) or the residual grows
    const int solver0 = h->local_solver;
    int fallback_at = -1;
    struct Restore {
        stokesmg* h;
        int s;
        ~Restore() { h->local_solver = s; }
    } restore{h, solver0};
    int64_t it0 = 0, so0 = 0;
    {
        unsigned long long c[2];
        SMG_HIP(h, hipMemcpyAsync(c, h->ws + h->cg_counter, sizeof(c), hipMemcpyDeviceToHost, st));
        SMG_HIP(h, hipStreamSynchronize(st));
        it0 = int64_t(c[0]);
        so0 = int64_t(c[1]);
    }

    double bnorm = 0.0;
    if (int rc = host_dots(h, b, 0, b, 1, N, &bnorm, st)) return rc;
    bnorm = std::sqrt(bnorm);
    SMG_HIP(h, smg::launch_zero(true, x, N, st));
    std::vector<double> hist{1.0};
    int it = 0;
    bool conv = bnorm == 0.0;
    std::vector<double> H(size_t(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), hv(restart + 1),
        h2(restart + 1);
    while (!conv && it < max_it) {
        // V_0 = r / |r|
        SMG_HIP(h, smg::launch_apply(k, true, true, x, b, V, tab64, n, st));
        double beta = 0.0;
        if (int rc = host_dots(h, V, 0, V, 1, N, &beta, st)) return rc;
        beta = std::sqrt(beta);
        if (beta / bnorm <= rtol) {
            conv = true;
            break;
        }
        SMG_HIP(h, smg::launch_multiaxpy(V, 0, coef, 0, 0.0, 1.0 / beta, V, N, st));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        for (int j = 0; j < restart; ++j) {
            double* vj = V + size_t(j) * N;
            // z_j = P^{-1} v_j (FP32 V-cycle: convert on entry and exit, the precision boundary; z_j
            // stays FP32 in the basis and its FP64 copy feeds the FP64 operator)
            double* zj64;
            if (f32) {
                SMG_HIP(h, smg::launch_convert(true, vj, vin, N, st));
                if (int rc = vcycle_level(h, L, false, vin, zvec(j), st, nullptr)) return rc;
                SMG_HIP(h, smg::launch_convert(false, zvec(j), z64, N, st));
                zj64 = z64;
            } else {
                zj64 = static_cast<double*>(zvec(j));
                if (int rc = vcycle_level(h, L, true, vj, zj64, st, nullptr)) return rc;
            }
            // w = K z_j, orthogonalized twice against V_0..V_j (classical Gram-Schmidt, twice)
            SMG_HIP(h, smg::launch_apply(k, true, false, zj64, nullptr, w, tab64, n, st));
            if (int rc = host_dots(h, V, N, w, j + 1, N, hv.data(), st)) return rc;
            SMG_HIP(h, hipMemcpyAsync(coef, hv.data(), (j + 1) * sizeof(double), hipMemcpyHostToDevice, st));
            SMG_HIP(h, smg::launch_multiaxpy(V, N, coef, j + 1, -1.0, 1.0, w, N, st));
            SMG_HIP(h, hipStreamSynchronize(st));
            if (int rc = host_dots(h, V, N, w, j + 1, N, h2.data(), st)) return rc;
            SMG_HIP(h, hipMemcpyAsync(coef, h2.data(), (j + 1) * sizeof(double), hipMemcpyHostToDevice, st));
            SMG_HIP(h, smg::launch_multiaxpy(V, N, coef, j + 1, -1.0, 1.0, w, N, st));
            SMG_HIP(h, hipStreamSynchronize(st));
            double hn = 0.0;
            if (int rc = host_dots(h, w, 0, w, 1, N, &hn, st)) return rc;
            bool finite = std::isfinite(hn);
            for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(hv[i]) && std::isfinite(h2[i]);
            if (!finite) {
                if (h->local_solver != STOKESMG_LOCAL_MLP)
                    return h->fail(STOKESMG_EHIP, "non-finite values in the preconditioned Krylov vector");
                // a non-finite learned correction: drop this step, restart with the exact local solver
                h->local_solver = STOKESMG_LOCAL_EXACT;
                fallback_at = it;
                break;
            }
            for (int i = 0; i <= j; ++i) H[size_t(i) * restart + j] = hv[i] + h2[i];
            hn = std::sqrt(hn);
            H[size_t(j + 1) * restart + j] = hn;
            double* vn = V + size_t(j + 1) * N;
            SMG_HIP(h, hipMemcpyAsync(vn, w, nb, hipMemcpyDeviceToDevice, st));
            if (hn > 0) SMG_HIP(h, smg::launch_multiaxpy(V, 0, coef, 0, 0.0, 1.0 / hn, vn, N, st));
            // Givens rotations
            for (int i = 0; i < j; ++i) {
                const double a = H[size_t(i) * restart + j], bb = H[size_t(i + 1) * restart + j];
                H[size_t(i) * restart + j] = cs[i] * a + sn[i] * bb;
                H[size_t(i + 1) * restart + j] = -sn[i] * a + cs[i] * bb;
            }
            const double a = H[size_t(j) * restart + j], bb = H[size_t(j + 1) * restart + j];
            const double den = std::hypot(a, bb);
            cs[j] = a / den;
            sn[j] = bb / den;
            H[size_t(j) * restart + j] = den;
            H[size_t(j + 1) * restart + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            jdone = j + 1;
            hist.push_back(std::fabs(g[j + 1]) / bnorm);
            if (h->local_solver == STOKESMG_LOCAL_MLP) {
                const double rho = hist[hist.size() - 1] / hist[hist.size() - 2];
                const double bound = h->rho_ref > 0.0 ? std::max(2.0 * h->rho_ref, 1e-3) : 1.0;
                if (!(rho < bound)) {   // also catches NaN
                    // keep this step, then restart: the Krylov directions of the learned
                    // steps would slow the exact ones down
                    h->local_solver = STOKESMG_LOCAL_EXACT;
                    fallback_at = it;
                    break;
                }
            }
            if (hist.back() <= rtol || it >= max_it) break;
        }
        // x += Z y, H(0:j, 0:j) y = g(0:j)
        if (jdone == 0) continue;
        std::vector<double> y(jdone);
        for (int i = jdone - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < jdone; ++q) s -= H[size_t(i) * restart + q] * y[q];
            y[i] = s / H[size_t(i) * restart + i];
        }
        SMG_HIP(h, hipMemcpyAsync(coef, y.data(), jdone * sizeof(double), hipMemcpyHostToDevice, st));
        if (f32) {
            for (int i = 0; i < jdone; ++i) {
                SMG_HIP(h, smg::launch_convert(false, zvec(i), z64, N, st));
                SMG_HIP(h, smg::launch_multiaxpy(z64, 0, coef + i, 1, 1.0, 1.0, x, N, st));
            }
        } else {
            SMG_HIP(h, smg::launch_multiaxpy(static_cast<const double*>(zvec(0)), N, coef, jdone, 1.0, 1.0, x, N, st));
        }
        SMG_HIP(h, hipStreamSynchronize(st));
        if (hist.back() <= rtol) conv = true;
    }
    // zero-mean pressure (L^2_0), then the true residual of the returned x
    SMG_HIP(h, smg::launch_normalize_pressure(true, x, h->lv[L].N1, k + 1,
                                              reinterpret_cast<const double*>(h->ws + h->wg_off), h->lv[L].h,
                                              reinterpret_cast<double*>(h->ws + h->scratch_off) + stokesmg::kMoment, st));
    SMG_HIP(h, smg::launch_apply(k, true, true, x, b, w, tab64, n, st));
    double rn = 0.0;
    if (int rc = host_dots(h, w, 0, w, 1, N, &rn, st)) return rc;
    const auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iterations = it;
        info->converged = conv ? 1 : 0;
        info->rel_residual = bnorm > 0 ? std::sqrt(rn) / bnorm : 0.0;
        const double last = hist.back();
        info->nu = (it > 0 && last > 0) ? -8.0 / (std::log10(last) / it) : 0.0;
        for (size_t i = 0; i < hist.size() && i < STOKESMG_MAX_HISTORY; ++i) info->history[i] = hist[i];
        unsigned long long c[2];
        SMG_HIP(h, hipMemcpyAsync(c, h->ws + h->cg_counter, sizeof(c), hipMemcpyDeviceToHost, st));
        SMG_HIP(h, hipStreamSynchronize(st));
        info->cg_iterations = int64_t(c[0]) - it0;
        info->local_solves = int64_t(c[1]) - so0;
        info->seconds = std::chrono::duration<double>(t1 - t0).count();
        info->fallback_iteration = fallback_at;
    }
    return conv ? STOKESMG_OK : h->fail(STOKESMG_ENOTCONV, "FGMRES reached max_it");
}

int stokesmg_rhs_manufactured(stokesmg_t* h, int level, int problem, double* b, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (level < 0 || level >= h->n_levels || !b) return h->fail(STOKESMG_EINVAL, "bad level or null vector");
    if (problem != STOKESMG_PROBLEM_SINE) return h->fail(STOKESMG_EINVAL, "unknown problem");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto& lv = h->lv[level];
    const int n = lv.n, N1 = lv.N1;
    smg::Ref1D ref(h->cfg.k);
    const double P = M_PI, P3 = 3.0 * P * P * P;
    // f = 3 pi^2 u + grad p and the tangential trace g = u (curl of psi (1,1,1), p = cos cos cos)
    const std::vector<Term> f[3] = {
        {{P3, {SINPI, COSPI, SINPI}}, {-P3, {SINPI, SINPI, COSPI}}, {-P, {SINPI, COSPI, COSPI}}},
        {{P3, {SINPI, SINPI, COSPI}}, {-P3, {COSPI, SINPI, SINPI}}, {-P, {COSPI, SINPI, COSPI}}},
        {{P3, {COSPI, SINPI, SINPI}}, {-P3, {SINPI, COSPI, SINPI}}, {-P, {COSPI, COSPI, SINPI}}}};
    const std::vector<Term> u[3] = {{{P, {SINPI, COSPI, SINPI}}, {-P, {SINPI, SINPI, COSPI}}},
                                    {{P, {SINPI, SINPI, COSPI}}, {-P, {COSPI, SINPI, SINPI}}},
                                    {{P, {COSPI, SINPI, SINPI}}, {-P, {SINPI, COSPI, SINPI}}}};
    std::vector<double> out(size_t(level_total(h, level)), 0.0);
    const size_t nc = size_t(N1 - 1) * N1 * N1;
    for (int c = 0; c < 3; ++c) {
        const int ext[3] = {c == 0 ? N1 - 1 : N1, c == 1 ? N1 - 1 : N1, c == 2 ? N1 - 1 : N1};
        auto add = [&](double coef, const std::vector<double>& a0, const std::vector<double>& a1,
                       const std::vector<double>& a2) {
            for (int Zi = 0; Zi < ext[2]; ++Zi)
                for (int Yi = 0; Yi < ext[1]; ++Yi) {
                    const double s = coef * a1[Yi] * a2[Zi];
                    if (s == 0.0) continue;
                    double* row = out.data() + size_t(c) * nc + size_t(ext[0]) * (Yi + size_t(ext[1]) * Zi);
                    for (int Xi = 0; Xi < ext[0]; ++Xi) row[Xi] += s * a0[Xi];
                }
        };
        for (const auto& t : f[c]) {
            std::vector<double> v[3], bd[3];
            for (int d = 0; d < 3; ++d) load_1d(ref, n, d == c, [&](double x) { return fn(t.g[d], x); }, lv.gamma, v[d], bd[d]);
            add(t.c, v[0], v[1], v[2]);
        }
        // boundary (Nitsche) terms of the tangential data: faces normal to d != c
        for (const auto& t : u[c]) {
            std::vector<double> v[3], bd[3];
            for (int d = 0; d < 3; ++d) load_1d(ref, n, d == c, [&](double x) { return fn(t.g[d], x); }, lv.gamma, v[d], bd[d]);
            for (int d = 0; d < 3; ++d) {
                if (d == c) continue;
                // face integral: the other two directions by quadrature, direction d by the end values
                std::vector<double> a[3] = {v[0], v[1], v[2]};
                a[d] = bd[d];
                add(t.c, a[0], a[1], a[2]);
            }
        }
    }
    SMG_HIP(h, hipMemcpyAsync(b, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, st));
    SMG_HIP(h, hipStreamSynchronize(st));
    return STOKESMG_OK;
}

int stokesmg_rhs_fourier(stokesmg_t* h, int level, int n_modes, const int* kappa, const double* amp,
                         const double* theta, double* b, void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (level < 0 || level >= h->n_levels || !b) return h->fail(STOKESMG_EINVAL, "bad level or null vector");
    if (n_modes < 0 || (n_modes > 0 && (!kappa || !amp || !theta)))
        return h->fail(STOKESMG_EINVAL, "bad mode arrays");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto& lv = h->lv[level];
    const int n = lv.n, N1 = lv.N1;
    smg::Ref1D ref(h->cfg.k);
    std::vector<double> out(size_t(level_total(h, level)), 0.0);
    const size_t nc = size_t(N1 - 1) * N1 * N1;
    // cos(A + B + C + theta) with A = pi k0 x, B = pi k1 y, C = pi k2 z, expanded into the
    // eight separable products of cosines and sines of A, B, C
    for (int c = 0; c < 3; ++c) {
        const int ext[3] = {c == 0 ? N1 - 1 : N1, c == 1 ? N1 - 1 : N1, c == 2 ? N1 - 1 : N1};
        for (int m = 0; m < n_modes; ++m) {
            const int* kp = kappa + (size_t(c) * n_modes + m) * 3;
            const double a = amp[size_t(c) * n_modes + m], th = theta[size_t(c) * n_modes + m];
            std::vector<double> vc[3], vs[3], bd;
            for (int d = 0; d < 3; ++d) {
                const double w = M_PI * kp[d];
                load_1d(ref, n, d == c, [w](double x) { return std::cos(w * x); }, lv.gamma, vc[d], bd);
                load_1d(ref, n, d == c, [w](double x) { return std::sin(w * x); }, lv.gamma, vs[d], bd);
            }
            const double ct = a * std::cos(th), stt = a * std::sin(th);
            // (sA, sB, sC) selects sine factors; cos(phi) and sin(phi) coefficients of each product
            for (int sel = 0; sel < 8; ++sel) {
                const int ns = (sel & 1) + ((sel >> 1) & 1) + ((sel >> 2) & 1);
                // cos(phi) = sum over even ns of (-1)^(ns/2) prod; sin(phi) = sum over odd ns of (-1)^((ns-1)/2) prod
                const double coef = (ns % 2 == 0) ? ct * ((ns / 2) % 2 ? -1.0 : 1.0)
                                                  : -stt * (((ns - 1) / 2) % 2 ? -1.0 : 1.0);
                const std::vector<double>& a0 = (sel & 1) ? vs[0] : vc[0];
                const std::vector<double>& a1 = (sel & 2) ? vs[1] : vc[1];
                const std::vector<double>& a2 = (sel & 4) ? vs[2] : vc[2];
                for (int Zi = 0; Zi < ext[2]; ++Zi)
                    for (int Yi = 0; Yi < ext[1]; ++Yi) {
                        const double sc = coef * a1[Yi] * a2[Zi];
                        double* row = out.data() + size_t(c) * nc + size_t(ext[0]) * (Yi + size_t(ext[1]) * Zi);
                        for (int Xi = 0; Xi < ext[0]; ++Xi) row[Xi] += sc * a0[Xi];
                    }
            }
        }
    }
    SMG_HIP(h, hipMemcpyAsync(b, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, st));
    SMG_HIP(h, hipStreamSynchronize(st));
    return STOKESMG_OK;
}

}  // extern "C"
