// Host construction of the per-level stencil tables (FP64).
#include "tables.hpp"

#include <cmath>
#include <random>
#include <stdexcept>

#include "stencil_tables.hpp"

namespace smg {

namespace {

// Largest |y_table - y_dense| / max|y_dense| over a random vector: row r of
// the dense matrix against the table row of its position.  The table row's
// column o sits at (rel ? r : cell*m) + shift + o.
double check_rows(const Dense& Mat, int m, int width, int shift, bool rel, bool by_variant, int n,
                  const double* tab_base, int var_stride) {
    std::mt19937_64 g(12345);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    std::vector<double> x(Mat.cols);
    for (auto& v : x) v = U(g);
    double err = 0.0, mx = 0.0;
    for (int r = 0; r < Mat.rows; ++r) {
        double yd = 0.0;
        for (int c = 0; c < Mat.cols; ++c) yd += Mat(r, c) * x[c];
        const int cell = r / m, a = r % m;
        const double* row = tab_base + (by_variant ? var_stride * ld_variant(cell, n) : 0) + a * width;
        double yt = 0.0;
        for (int o = 0; o < width; ++o) {
            int c = (rel ? r : cell * m) + shift + o;
            if (c >= 0 && c < Mat.cols) yt += row[o] * x[c];
        }
        err = std::fmax(err, std::fabs(yt - yd));
        mx = std::fmax(mx, std::fabs(yd));
    }
    return err / (mx > 0 ? mx : 1.0);
}

}  // namespace

LevelTables build_level_tables(const Ref1D& r, int n, double penalty_factor) {
    const int k = r.k, m = k + 1;
    LevelTables T;
    T.n = n;
    T.k = k;
    T.N1 = n * m;
    T.h = 1.0 / n;
    T.gamma = penalty_factor * m * m / T.h;
    const double h = T.h;
    const int sz = tab_size(k);
    T.stencil.assign(sz, 0.0);
    double* t = T.stencil.data();
    const int oMC = 0, oLC = m * (2 * m + 1), oDT = 2 * m * (2 * m + 1), oDD = oDT + 2 * m * m,
              oLD = oDD + m * (m + 1), oMD = oLD + 12 * m * m;

    // continuous rows: position b of a cell is node j = b + 1 of the cell
    for (int b = 0; b < m; ++b) {
        const int j = b + 1;
        for (int jj = 0; jj <= m; ++jj) {                 // own cell's nodes: offset jj - j
            const int o = jj - j + m;
            t[oMC + b * (2 * m + 1) + o] += h * r.Mc(j, jj);
            t[oLC + b * (2 * m + 1) + o] += r.Kc(j, jj) / h;
        }
        if (j == m) {                                     // shared node: the next cell's nodes
            for (int jj = 0; jj <= m; ++jj) {
                const int o = m + jj;
                t[oMC + b * (2 * m + 1) + o] += h * r.Mc(0, jj);
                t[oLC + b * (2 * m + 1) + o] += r.Kc(0, jj) / h;
            }
        }
        for (int a = 0; a < m; ++a) {
            t[oDT + b * 2 * m + a] = r.D(a, j);
            if (j == m) t[oDT + b * 2 * m + m + a] = r.D(a, 0);
        }
    }
    for (int a = 0; a < m; ++a)
        for (int j = 0; j <= m; ++j) t[oDD + a * (m + 1) + j] = r.D(a, j);
    for (int a = 0; a < m; ++a) t[oMD + a] = h * r.wg[a];

    // DG rows: read off small assemblies with the level's h
    {
        Global1D g3(r, 3, h, penalty_factor), g1(r, 1, h, penalty_factor);
        const int src_cell[4] = {1, 0, 2, 0};
        for (int v = 0; v < 4; ++v) {
            const Global1D& g = (v == 3) ? g1 : g3;
            const int c = src_cell[v];
            for (int a = 0; a < m; ++a)
                for (int o = 0; o < 3 * m; ++o) {
                    const int col = c * m - m + o;
                    if (col >= 0 && col < g.N1)
                        t[oLD + v * 3 * m * m + a * 3 * m + o] = g.Ld(c * m + a, col);
                }
        }
    }

    // self-check against the directly assembled 1D matrices of this level
    Global1D G(r, n, h, penalty_factor);
    double e = 0.0;
    e = std::fmax(e, check_rows(G.Mc, m, 2 * m + 1, -m, true, false, n, t + oMC, 0));
    e = std::fmax(e, check_rows(G.Lc, m, 2 * m + 1, -m, true, false, n, t + oLC, 0));
    e = std::fmax(e, check_rows(G.Ld, m, 3 * m, -m, false, true, n, t + oLD, 3 * m * m));
    e = std::fmax(e, check_rows(G.D, m, m + 1, -1, false, false, n, t + oDD, 0));
    {
        // D^T rows (continuous position rows, pressure columns)
        Dense DTm(G.D.cols, G.D.rows);
        for (int i = 0; i < G.D.rows; ++i)
            for (int j = 0; j < G.D.cols; ++j) DTm(j, i) = G.D(i, j);
        e = std::fmax(e, check_rows(DTm, m, 2 * m, 0, false, false, n, t + oDT, 0));
    }
    for (int i = 0; i < T.N1; ++i) {
        double d = G.Md(i, i);
        e = std::fmax(e, std::fabs(d - t[oMD + i % m]) / std::fabs(d));
    }
    if (!(e < 1e-12))
        throw std::runtime_error("stencil table self-check failed for n=" + std::to_string(n) +
                                 " k=" + std::to_string(k) + " (rel err " + std::to_string(e) + ")");
    return T;
}

}  // namespace smg

// ------------------------------------------------------------------ patches
#include "eig.hpp"
#include "patch_tables.hpp"

namespace smg {

std::vector<double> build_patch_tables(const Ref1D& r, int n, double penalty_factor) {
    if (n < 2) return {};
    const int k = r.k, m = k + 1, nc = 2 * k + 1, nd = 2 * k + 2;
    const double h = 1.0 / n;
    std::vector<double> t(patch_tab_size(k), 0.0);
    const int oSC = 0, oLC = nc * nc, oSD = oLC + nc, oLD = oSD + 4 * nd * nd, oDP = oLD + 4 * nd,
              oMD = oDP + nd * nc;
    auto check = [&](const Dense& L, const Dense& M, const std::vector<double>& lam, const Dense& S) {
        const int q = L.rows;
        double e = 0.0, sc = 0.0;
        for (int i = 0; i < q; ++i) sc = std::fmax(sc, std::fabs(lam[i]));
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                double sm = 0.0, sl = 0.0;
                for (int a = 0; a < q; ++a)
                    for (int b = 0; b < q; ++b) {
                        sm += S(a, i) * M(a, b) * S(b, j);
                        sl += S(a, i) * L(a, b) * S(b, j);
                    }
                e = std::fmax(e, std::fabs(sm - (i == j ? 1.0 : 0.0)));
                e = std::fmax(e, std::fabs(sl - (i == j ? lam[i] : 0.0)) / sc);
            }
        if (!(e < 1e-9)) throw std::runtime_error("patch eigen-decomposition self-check failed");
    };
    // continuous window: interior nodes of two cells; identical for every patch
    {
        Global1D g(r, 4, h, penalty_factor);
        const int base = m;   // nodes of cells 1, 2 (interior-node indexing starts at g = 1)
        Dense L(nc, nc), M(nc, nc);
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nc; ++j) {
                L(i, j) = g.Lc(base + i, base + j);
                M(i, j) = g.Mc(base + i, base + j);
            }
        std::vector<double> lam;
        Dense S;
        generalized_eig(L, M, lam, S);
        check(L, M, lam, S);
        for (int i = 0; i < nc; ++i) {
            t[oLC + i] = lam[i];
            for (int j = 0; j < nc; ++j) t[oSC + i * nc + j] = S(i, j);
        }
        for (int i = 0; i < nd; ++i)
            for (int j = 0; j < nc; ++j) t[oDP + i * nc + j] = g.D(base + i, base + j);
    }
    // discontinuous windows: 4 boundary types
    {
        Global1D g4(r, 4, h, penalty_factor), g2(r, 2, h, penalty_factor);
        const Global1D* src[4] = {&g4, &g4, &g4, &g2};
        const int base[4] = {m, 0, 2 * m, 0};
        for (int ty = 0; ty < 4; ++ty) {
            Dense L(nd, nd), M(nd, nd);
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nd; ++j) {
                    L(i, j) = src[ty]->Ld(base[ty] + i, base[ty] + j);
                    M(i, j) = src[ty]->Md(base[ty] + i, base[ty] + j);
                }
            std::vector<double> lam;
            Dense S;
            generalized_eig(L, M, lam, S);
            check(L, M, lam, S);
            for (int i = 0; i < nd; ++i) {
                t[oLD + ty * nd + i] = lam[i];
                for (int j = 0; j < nd; ++j) t[oSD + ty * nd * nd + i * nd + j] = S(i, j);
            }
        }
    }
    for (int i = 0; i < nd; ++i) t[oMD + i] = h * r.wg[i % m];
    return t;
}

}  // namespace smg
