// 1D finite element data for RT_k x DG Q_k on Cartesian cells (host, FP64).
//
// The Raviart-Thomas element of Sec. 2.1 is a tensor product of 1D spaces:
// degree k+1 in a component's own ("parallel") direction, where the normal
// component is continuous, and degree k in the "orthogonal" directions
// (Fig. RT2 and the text around it).  Nodal bases: Lagrange polynomials on
// the k+2 Gauss-Lobatto points (continuous direction) and on the k+1 Gauss
// points (discontinuous directions, pressure).  With these the DG mass is
// diagonal, h * w_a, and the operator of Eq. bilinear separates into the 1D
// matrices built here (the Kronecker structure named in Sec. 2.2).
#pragma once

#include <cmath>
#include <stdexcept>
#include <vector>

namespace smg {

struct Dense {
    int rows = 0, cols = 0;
    std::vector<double> a;
    Dense() = default;
    Dense(int r, int c) : rows(r), cols(c), a(size_t(r) * c, 0.0) {}
    double& operator()(int i, int j) { return a[size_t(i) * cols + j]; }
    double operator()(int i, int j) const { return a[size_t(i) * cols + j]; }
};

// Legendre polynomial P_n and its derivative on [-1, 1] (three-term recurrence).
inline void legendre(int n, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    // P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1), valid off the endpoints
    dp = n * (x * p1 - p0) / (x * x - 1.0);
}

// Gauss-Legendre points and weights on [0, 1], Newton iteration on P_n.
inline void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, t, p, dp);
            double dt = p / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        double p, dp;
        legendre(n, t, p, dp);
        x[n - 1 - i] = 0.5 * (t + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);   // 2/((1-t^2)P'^2) scaled by 1/2
    }
}

// Gauss-Lobatto points (n >= 2, endpoints included) on [0, 1]: the interior
// points are the roots of P'_{n-1}; Newton with P''_{n-1} from the Legendre
// equation (1 - t^2) P'' = 2 t P' - N (N + 1) P.
inline std::vector<double> gauss_lobatto_points(int n) {
    std::vector<double> x(n);
    const int N = n - 1;
    x[0] = 0.0;
    x[n - 1] = 1.0;
    for (int i = 1; i < n - 1; ++i) {
        double t = -std::cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, t, p, dp);
            double ddp = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
            double dt = dp / ddp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        x[i] = 0.5 * (t + 1.0);
    }
    return x;
}

inline double lagrange(const std::vector<double>& nodes, int i, double x) {
    double v = 1.0;
    for (size_t j = 0; j < nodes.size(); ++j)
        if (int(j) != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    return v;
}

inline double lagrange_deriv(const std::vector<double>& nodes, int i, double x) {
    double s = 0.0;
    for (size_t r = 0; r < nodes.size(); ++r) {
        if (int(r) == i) continue;
        double t = 1.0 / (nodes[i] - nodes[r]);
        for (size_t j = 0; j < nodes.size(); ++j)
            if (int(j) != i && j != r) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
        s += t;
    }
    return s;
}

// Reference (h = 1) 1D matrices of one cell, integrated exactly by the
// (k+2)-point Gauss rule.
struct Ref1D {
    int k = 0;
    std::vector<double> xg, wg;   // Gauss nodes/weights (DG basis), k+1
    std::vector<double> xl;       // Gauss-Lobatto nodes (continuous basis), k+2
    Dense Md, Kd;                 // (k+1)^2: int l_a l_b, int l_a' l_b'
    Dense Mc, Kc;                 // (k+2)^2: int phi_a phi_b, int phi_a' phi_b'
    Dense D;                      // (k+1) x (k+2): int l_a phi_b'
    std::vector<double> eL, eR, dL, dR;   // l_a(0), l_a(1), l_a'(0), l_a'(1)

    explicit Ref1D(int k_) : k(k_) {
        if (k < 1 || k > 5) throw std::invalid_argument("degree must be 1..5");
        const int m = k + 1;
        gauss_rule(m, xg, wg);
        xl = gauss_lobatto_points(m + 1);
        std::vector<double> xq, wq;
        gauss_rule(k + 2, xq, wq);
        Md = Dense(m, m); Kd = Dense(m, m);
        Mc = Dense(m + 1, m + 1); Kc = Dense(m + 1, m + 1);
        D = Dense(m, m + 1);
        for (size_t q = 0; q < xq.size(); ++q) {
            for (int a = 0; a < m; ++a) {
                double la = lagrange(xg, a, xq[q]), da = lagrange_deriv(xg, a, xq[q]);
                for (int b = 0; b < m; ++b) {
                    Md(a, b) += wq[q] * la * lagrange(xg, b, xq[q]);
                    Kd(a, b) += wq[q] * da * lagrange_deriv(xg, b, xq[q]);
                }
                for (int b = 0; b <= m; ++b) D(a, b) += wq[q] * la * lagrange_deriv(xl, b, xq[q]);
            }
            for (int a = 0; a <= m; ++a) {
                double pa = lagrange(xl, a, xq[q]), dpa = lagrange_deriv(xl, a, xq[q]);
                for (int b = 0; b <= m; ++b) {
                    Mc(a, b) += wq[q] * pa * lagrange(xl, b, xq[q]);
                    Kc(a, b) += wq[q] * dpa * lagrange_deriv(xl, b, xq[q]);
                }
            }
        }
        for (int a = 0; a < m; ++a) {
            eL.push_back(lagrange(xg, a, 0.0));
            eR.push_back(lagrange(xg, a, 1.0));
            dL.push_back(lagrange_deriv(xg, a, 0.0));
            dR.push_back(lagrange_deriv(xg, a, 1.0));
        }
    }
};

// Global 1D matrices of one direction on n cells (h = 1/n), assembled
// directly: the 1D restriction of Eq. bilinear on the DG side (cell
// stiffness, interior-face terms gamma [u][v] - {{u'}}[v] - [u]{{v'}} and
// boundary terms 2 gamma u v - d_n u v - u d_n v), and stiffness/mass with
// shared nodes on the continuous side (restricted to the interior nodes:
// the boundary normal nodes are eliminated, Sec. 2.1).
struct Global1D {
    int n = 0, k = 0, N1 = 0;
    double h = 0, gamma = 0;
    Dense Md, Ld;      // N1 x N1
    Dense Mc, Lc;      // (N1-1) x (N1-1), interior nodes g = 1..N1-1
    Dense D;           // N1 x (N1-1): int psi_q phi_g'

    // n_ cells of width h_ (h_ = 1/n_ for a level of the unit cube; other
    // values serve to extract the rows of a level from a few cells).
    Global1D(const Ref1D& r, int n_, double h_, double penalty_factor) : n(n_), k(r.k) {
        const int m = k + 1;
        N1 = n * m;
        h = h_;
        gamma = penalty_factor * m * m / h;
        Md = Dense(N1, N1); Ld = Dense(N1, N1);
        Dense McF(N1 + 1, N1 + 1), LcF(N1 + 1, N1 + 1), DF(N1, N1 + 1);
        for (int c = 0; c < n; ++c) {
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b) {
                    Md(c * m + a, c * m + b) += h * r.Md(a, b);
                    Ld(c * m + a, c * m + b) += r.Kd(a, b) / h;
                }
            for (int a = 0; a <= m; ++a) {
                for (int b = 0; b <= m; ++b) {
                    McF(c * m + a, c * m + b) += h * r.Mc(a, b);
                    LcF(c * m + a, c * m + b) += r.Kc(a, b) / h;
                }
            }
            for (int a = 0; a < m; ++a)
                for (int b = 0; b <= m; ++b) DF(c * m + a, c * m + b) += r.D(a, b);
        }
        // face terms on the DG side; trial u (column), test v (row)
        std::vector<double> J(N1), A(N1);
        for (int f = 1; f < n; ++f) {       // face between cell f-1 (minus side) and cell f
            std::fill(J.begin(), J.end(), 0.0);
            std::fill(A.begin(), A.end(), 0.0);
            for (int a = 0; a < m; ++a) {
                J[(f - 1) * m + a] += r.eR[a];
                J[f * m + a] -= r.eL[a];
                A[(f - 1) * m + a] += 0.5 * r.dR[a] / h;
                A[f * m + a] += 0.5 * r.dL[a] / h;
            }
            for (int i = 0; i < N1; ++i)
                for (int j = 0; j < N1; ++j)
                    Ld(i, j) += gamma * J[i] * J[j] - J[i] * A[j] - A[i] * J[j];
        }
        for (int side = 0; side < 2; ++side) {
            std::fill(J.begin(), J.end(), 0.0);
            std::fill(A.begin(), A.end(), 0.0);
            for (int a = 0; a < m; ++a) {
                if (side == 0) { J[a] = r.eL[a]; A[a] = -r.dL[a] / h; }     // outward normal -1
                else { J[(n - 1) * m + a] = r.eR[a]; A[(n - 1) * m + a] = r.dR[a] / h; }
            }
            for (int i = 0; i < N1; ++i)
                for (int j = 0; j < N1; ++j)
                    Ld(i, j) += 2.0 * gamma * J[i] * J[j] - J[i] * A[j] - A[i] * J[j];
        }
        Mc = Dense(N1 - 1, N1 - 1); Lc = Dense(N1 - 1, N1 - 1); D = Dense(N1, N1 - 1);
        for (int i = 1; i < N1; ++i)
            for (int j = 1; j < N1; ++j) {
                Mc(i - 1, j - 1) = McF(i, j);
                Lc(i - 1, j - 1) = LcF(i, j);
            }
        for (int q = 0; q < N1; ++q)
            for (int g = 1; g < N1; ++g) D(q, g - 1) = DF(q, g);
    }
};

}  // namespace smg
