// Host construction of the multigrid data (FP64).
#include "mg_tables.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace smg {

namespace {

Rows1D transpose(const Rows1D& a, int cols) {
    std::vector<std::vector<std::pair<int, double>>> lists(cols);
    for (int i = 0; i < a.rows; ++i)
        for (int t = 0; t < a.width; ++t) {
            const int j = a.idx[size_t(i) * a.width + t];
            if (j >= 0) lists[j].push_back({i, a.w[size_t(i) * a.width + t]});
        }
    Rows1D out;
    out.rows = cols;
    out.width = 1;
    for (auto& l : lists) out.width = std::max<int>(out.width, int(l.size()));
    out.idx.assign(size_t(cols) * out.width, -1);
    out.w.assign(size_t(cols) * out.width, 0.0);
    for (int j = 0; j < cols; ++j)
        for (size_t t = 0; t < lists[j].size(); ++t) {
            out.idx[size_t(j) * out.width + t] = lists[j][t].first;
            out.w[size_t(j) * out.width + t] = lists[j][t].second;
        }
    return out;
}

}  // namespace

Transfer1D build_transfer(const Ref1D& r, int nc) {
    const int k = r.k, m = k + 1, nf = 2 * nc;
    const int N1c = nc * m, N1f = nf * m;
    Transfer1D T;
    // DG: fine position (cell f, a) lies in coarse cell f/2 at (child + x_a)/2
    T.pd.rows = N1f;
    T.pd.width = m;
    T.pd.idx.resize(size_t(N1f) * m);
    T.pd.w.resize(size_t(N1f) * m);
    for (int X = 0; X < N1f; ++X) {
        const int f = X / m, a = X % m, C = f / 2, child = f % 2;
        const double xi = 0.5 * (child + r.xg[a]);
        for (int b = 0; b < m; ++b) {
            T.pd.idx[size_t(X) * m + b] = C * m + b;
            T.pd.w[size_t(X) * m + b] = lagrange(r.xg, b, xi);
        }
    }
    // continuous: fine interior node g = f m + j (j = 0..m-1 with x = (f + xl_j) h_f)
    T.pc.rows = N1f - 1;
    T.pc.width = m + 1;
    T.pc.idx.assign(size_t(N1f - 1) * (m + 1), -1);
    T.pc.w.assign(size_t(N1f - 1) * (m + 1), 0.0);
    for (int X = 0; X < N1f - 1; ++X) {
        const int g = X + 1, f = g / m, j = g % m;
        const double xf = (f + r.xl[j]) / nf;              // physical coordinate
        int C = int(std::floor(xf * nc));
        C = std::min(std::max(C, 0), nc - 1);
        const double xi = xf * nc - C;
        for (int b = 0; b <= m; ++b) {
            const int gc = C * m + b;
            if (gc < 1 || gc > N1c - 1) continue;         // eliminated boundary node
            const double v = lagrange(r.xl, b, xi);
            if (v == 0.0) continue;
            T.pc.idx[size_t(X) * (m + 1) + b] = gc - 1;
            T.pc.w[size_t(X) * (m + 1) + b] = v;
        }
    }
    T.rd = transpose(T.pd, N1c);
    T.rc = transpose(T.pc, N1c - 1);
    return T;
}

std::vector<double> coarse_pseudo_inverse(const Ref1D& r, int n0, double penalty_factor, int* N0_out) {
    Global1D g(r, n0, 1.0 / n0, penalty_factor);
    const int N1 = g.N1, Nc = N1 - 1;
    const int nc = Nc * N1 * N1, np = N1 * N1 * N1, N = 3 * nc + np;
    // factor matrices for x-fastest storage: entry of kron(Z, Y, X) at
    // ((z, y, x), (z', y', x')) = Z(z, z') Y(y, y') X(x, x')
    auto kron3_add = [&](std::vector<double>& K, int ro, int co, const Dense& Zm, const Dense& Ym, const Dense& Xm,
                         double s) {
        for (int z = 0; z < Zm.rows; ++z)
            for (int y = 0; y < Ym.rows; ++y)
                for (int x = 0; x < Xm.rows; ++x) {
                    const int row = ro + x + Xm.rows * (y + Ym.rows * z);
                    for (int z2 = 0; z2 < Zm.cols; ++z2) {
                        const double zz = Zm(z, z2);
                        if (zz == 0.0) continue;
                        for (int y2 = 0; y2 < Ym.cols; ++y2) {
                            const double yy = zz * Ym(y, y2);
                            if (yy == 0.0) continue;
                            for (int x2 = 0; x2 < Xm.cols; ++x2) {
                                const int col = co + x2 + Xm.cols * (y2 + Ym.cols * z2);
                                K[size_t(row) * N + col] += s * yy * Xm(x, x2);
                            }
                        }
                    }
                }
    };
    std::vector<double> K(size_t(N) * N, 0.0);
    const Dense &Md = g.Md, &Ld = g.Ld, &Mc = g.Mc, &Lc = g.Lc, &D = g.D;
    // A_x, A_y, A_z (factors in (z, y, x) order for kron)
    kron3_add(K, 0, 0, Md, Md, Lc, 1.0);
    kron3_add(K, 0, 0, Md, Ld, Mc, 1.0);
    kron3_add(K, 0, 0, Ld, Md, Mc, 1.0);
    kron3_add(K, nc, nc, Md, Lc, Md, 1.0);
    kron3_add(K, nc, nc, Md, Mc, Ld, 1.0);
    kron3_add(K, nc, nc, Ld, Mc, Md, 1.0);
    kron3_add(K, 2 * nc, 2 * nc, Lc, Md, Md, 1.0);
    kron3_add(K, 2 * nc, 2 * nc, Mc, Ld, Md, 1.0);
    kron3_add(K, 2 * nc, 2 * nc, Mc, Md, Ld, 1.0);
    // B = -[D Md Md | Md D Md | Md Md D] and B^T
    kron3_add(K, 3 * nc, 0, Md, Md, D, -1.0);
    kron3_add(K, 3 * nc, nc, Md, D, Md, -1.0);
    kron3_add(K, 3 * nc, 2 * nc, D, Md, Md, -1.0);
    for (int i = 3 * nc; i < N; ++i)
        for (int j = 0; j < 3 * nc; ++j) K[size_t(j) * N + i] = K[size_t(i) * N + j];
    // bordered system and its inverse by Gauss-Jordan with partial pivoting
    const int Nb = N + 1;
    std::vector<double> A(size_t(Nb) * Nb, 0.0), I(size_t(Nb) * Nb, 0.0);
    const double cval = 1.0 / std::sqrt(double(np));
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A[size_t(i) * Nb + j] = K[size_t(i) * N + j];
    for (int i = 3 * nc; i < N; ++i) A[size_t(i) * Nb + N] = A[size_t(N) * Nb + i] = cval;
    for (int i = 0; i < Nb; ++i) I[size_t(i) * Nb + i] = 1.0;
    for (int col = 0; col < Nb; ++col) {
        int piv = col;
        for (int i = col + 1; i < Nb; ++i)
            if (std::fabs(A[size_t(i) * Nb + col]) > std::fabs(A[size_t(piv) * Nb + col])) piv = i;
        if (std::fabs(A[size_t(piv) * Nb + col]) < 1e-300) throw std::runtime_error("bordered coarse matrix singular");
        if (piv != col)
            for (int j = 0; j < Nb; ++j) {
                std::swap(A[size_t(piv) * Nb + j], A[size_t(col) * Nb + j]);
                std::swap(I[size_t(piv) * Nb + j], I[size_t(col) * Nb + j]);
            }
        const double d = 1.0 / A[size_t(col) * Nb + col];
        for (int j = 0; j < Nb; ++j) {
            A[size_t(col) * Nb + j] *= d;
            I[size_t(col) * Nb + j] *= d;
        }
        for (int i = 0; i < Nb; ++i) {
            if (i == col) continue;
            const double f = A[size_t(i) * Nb + col];
            if (f == 0.0) continue;
            for (int j = 0; j < Nb; ++j) {
                A[size_t(i) * Nb + j] -= f * A[size_t(col) * Nb + j];
                I[size_t(i) * Nb + j] -= f * I[size_t(col) * Nb + j];
            }
        }
    }
    std::vector<double> P(size_t(N) * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) P[size_t(i) * N + j] = 0.5 * (I[size_t(i) * Nb + j] + I[size_t(j) * Nb + i]);
    // self-check: K P K = K
    double e = 0.0, sc = 0.0;
    std::vector<double> KP(size_t(N) * N, 0.0);
    for (int i = 0; i < N; ++i)
        for (int t = 0; t < N; ++t) {
            const double kit = K[size_t(i) * N + t];
            if (kit == 0.0) continue;
            for (int j = 0; j < N; ++j) KP[size_t(i) * N + j] += kit * P[size_t(t) * N + j];
        }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double v = 0.0;
            for (int t = 0; t < N; ++t) v += KP[size_t(i) * N + t] * K[size_t(t) * N + j];
            e = std::fmax(e, std::fabs(v - K[size_t(i) * N + j]));
            sc = std::fmax(sc, std::fabs(K[size_t(i) * N + j]));
        }
    if (!(e < 1e-9 * sc)) throw std::runtime_error("coarse pseudo-inverse self-check failed");
    *N0_out = N;
    return P;
}

}  // namespace smg
