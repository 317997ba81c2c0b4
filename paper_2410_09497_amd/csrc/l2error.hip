// L2 errors of a discrete solution against the built-in manufactured
// solution (Sec. 3.3 measures convergence and error against time; the
// survey's error-versus-time study): ||u - u_h|| and ||p - p_h|| over the unit
// cube with Gauss quadrature of k+3 points per direction in every cell, the
// pressures compared with zero integral mean.  One workgroup per cell at a
// time (grid-stride over cells); the cell's coefficients are staged in LDS
// and every quadrature point sums its basis expansion.  Partial sums per
// workgroup go to the workspace scratch and are added on the host in a fixed
// order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "handle.hpp"

namespace {

constexpr int kMaxQ = 8;          // k + 3 for k <= 5
constexpr int kThreads = 256;

struct L2Tab {
    int k, q, n, N1;
    double h;
    double xq[kMaxQ], wq[kMaxQ];
    double phi[kMaxQ - 1][kMaxQ];   // Gauss-Lobatto Lagrange basis j (k+2 nodes) at quadrature point a
    double psi[kMaxQ - 2][kMaxQ];   // Gauss Lagrange basis b (k+1 nodes) at quadrature point a
};

// the sine problem: u = curl(sin(pi x) sin(pi y) sin(pi z) (1,1,1)), p = cos cos cos
__device__ inline void sine_exact(double x, double y, double z, double* u) {
    const double sx = sinpi(x), sy = sinpi(y), sz = sinpi(z), cx = cospi(x), cy = cospi(y), cz = cospi(z);
    u[0] = M_PI * sx * (cy * sz - sy * cz);
    u[1] = M_PI * sy * (sx * cz - cx * sz);
    u[2] = M_PI * sz * (cx * sy - sx * cy);
    u[3] = cx * cy * cz;
}

__global__ void __launch_bounds__(kThreads) l2_error_kernel(const double* __restrict__ xv, L2Tab t,
                                                            double* __restrict__ partial) {
    __shared__ double coef[3 * 7 * 36 + 216];
    __shared__ double red[3][kThreads];
    const int m = t.k + 1, mc = t.k + 2, q = t.q, N1 = t.N1, n = t.n;
    const size_t nc = size_t(N1 - 1) * N1 * N1;
    const int nvc = mc * m * m;                 // coefficients of one velocity component in a cell
    const int ncell = nvc * 3 + m * m * m;
    double eu = 0.0, ep = 0.0, dp = 0.0;
    const long long cells = (long long)n * n * n;
    for (long long cell = blockIdx.x; cell < cells; cell += gridDim.x) {
        const int cx = int(cell % n), cy = int((cell / n) % n), cz = int(cell / ((long long)n * n));
        __syncthreads();
        for (int i = threadIdx.x; i < ncell; i += kThreads) {
            double v = 0.0;
            if (i < 3 * nvc) {
                const int c = i / nvc, e = i - c * nvc;
                // local (j, b, b') with j the continuous index of component c (its own direction)
                const int j = e % mc, r = e / mc, b1 = r % m, b2 = r / m;
                const int cc[3] = {cx, cy, cz};
                const int pos_c = cc[c] * m + j - 1;    // continuous position; -1 and N1 - 1 are boundary nodes
                const int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
                const int p1 = cc[d1] * m + b1, p2 = cc[d2] * m + b2;
                if (pos_c >= 0 && pos_c < N1 - 1) {
                    int P[3];
                    P[c] = pos_c;
                    P[d1] = p1;
                    P[d2] = p2;
                    size_t g;
                    if (c == 0) g = size_t(P[0]) + size_t(N1 - 1) * (P[1] + size_t(N1) * P[2]);
                    else if (c == 1) g = nc + P[0] + size_t(N1) * (P[1] + size_t(N1 - 1) * P[2]);
                    else g = 2 * nc + P[0] + size_t(N1) * (P[1] + size_t(N1) * P[2]);
                    v = xv[g];
                }
            } else {
                const int e = i - 3 * nvc;
                const int a0 = e % m, a1 = (e / m) % m, a2 = e / (m * m);
                v = xv[3 * nc + size_t(cx * m + a0) + size_t(N1) * (cy * m + a1 + size_t(N1) * (cz * m + a2))];
            }
            coef[i] = v;
        }
        __syncthreads();
        for (int pt = threadIdx.x; pt < q * q * q; pt += kThreads) {
            const int a = pt % q, b = (pt / q) % q, c = pt / (q * q);
            const int qa[3] = {a, b, c};
            double uh[4] = {0.0, 0.0, 0.0, 0.0};
            for (int comp = 0; comp < 3; ++comp) {
                const int d1 = (comp + 1) % 3, d2 = (comp + 2) % 3;
                const double* cf = coef + comp * nvc;
                double s = 0.0;
                for (int b2 = 0; b2 < m; ++b2)
                    for (int b1 = 0; b1 < m; ++b1) {
                        const double w12 = t.psi[b1][qa[d1]] * t.psi[b2][qa[d2]];
                        double sj = 0.0;
                        for (int j = 0; j < mc; ++j) sj += cf[j + mc * (b1 + m * b2)] * t.phi[j][qa[comp]];
                        s += w12 * sj;
                    }
                uh[comp] = s;
            }
            {
                const double* cf = coef + 3 * nvc;
                double s = 0.0;
                for (int a2 = 0; a2 < m; ++a2)
                    for (int a1 = 0; a1 < m; ++a1) {
                        const double w12 = t.psi[a1][b] * t.psi[a2][c];
                        double sj = 0.0;
                        for (int a0 = 0; a0 < m; ++a0) sj += cf[a0 + m * (a1 + m * a2)] * t.psi[a0][a];
                        s += w12 * sj;
                    }
                uh[3] = s;
            }
            double ue[4];
            sine_exact((cx + t.xq[a]) * t.h, (cy + t.xq[b]) * t.h, (cz + t.xq[c]) * t.h, ue);
            const double w = t.wq[a] * t.wq[b] * t.wq[c] * t.h * t.h * t.h;
            for (int comp = 0; comp < 3; ++comp) eu += w * (uh[comp] - ue[comp]) * (uh[comp] - ue[comp]);
            const double e = uh[3] - ue[3];
            ep += w * e * e;
            dp += w * e;
        }
    }
    red[0][threadIdx.x] = eu;
    red[1][threadIdx.x] = ep;
    red[2][threadIdx.x] = dp;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int r = 0; r < 3; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int r = 0; r < 3; ++r) partial[3 * blockIdx.x + r] = red[r][0];
}

}  // namespace

extern "C" {

int stokesmg_l2_error(stokesmg_t* h, int level, int problem, const double* x, double* err_u, double* err_p,
                      void* stream) {
    if (!h) return STOKESMG_EINVAL;
    if (level < 0 || level >= h->n_levels || !x || !err_u || !err_p)
        return h->fail(STOKESMG_EINVAL, "bad level or null pointer");
    if (problem != STOKESMG_PROBLEM_SINE) return h->fail(STOKESMG_EINVAL, "unknown problem");
    if (!h->ws) return h->fail(STOKESMG_ENOMEM, "no workspace set");
    const int k = h->cfg.k;
    L2Tab t{};
    t.k = k;
    t.q = k + 3;
    t.n = h->lv[level].n;
    t.N1 = h->lv[level].N1;
    t.h = h->lv[level].h;
    smg::Ref1D ref(k);
    std::vector<double> xq, wq;
    smg::gauss_rule(t.q, xq, wq);
    for (int a = 0; a < t.q; ++a) {
        t.xq[a] = xq[a];
        t.wq[a] = wq[a];
        for (int j = 0; j < k + 2; ++j) t.phi[j][a] = smg::lagrange(ref.xl, j, xq[a]);
        for (int b = 0; b < k + 1; ++b) t.psi[b][a] = smg::lagrange(ref.xg, b, xq[a]);
    }
    const int blocks = stokesmg::kPartialBlocks;
    double* partial = reinterpret_cast<double*>(h->ws + h->scratch_off) + stokesmg::kPartial;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(l2_error_kernel, dim3(blocks), dim3(kThreads), 0, st, x, t, partial);
    SMG_HIP(h, hipGetLastError());
    std::vector<double> p(size_t(3) * blocks);
    SMG_HIP(h, hipMemcpyAsync(p.data(), partial, p.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    SMG_HIP(h, hipStreamSynchronize(st));
    double eu = 0.0, ep = 0.0, dp = 0.0;
    for (int b = 0; b < blocks; ++b) {
        eu += p[3 * b];
        ep += p[3 * b + 1];
        dp += p[3 * b + 2];
    }
    *err_u = std::sqrt(eu);
    *err_p = std::sqrt(std::fmax(ep - dp * dp, 0.0));   // pressures with zero mean (unit volume)
    return STOKESMG_OK;
}

}  // extern "C"
