// The "Direct" local solver of Sec. 3.3 (the pseudo-inverse of the patch
// matrix) for interior patches, as one dense matrix per degree.
//
// An interior patch (its 8 cells touch no boundary face) has the patch matrix
// K_j(h) = [[h A^, h^2 B^T], [h^2 B^, 0]] with level-independent A^, B^ (A_j
// scales like h, B_j like h^2).  In the normalized variables of the patch
// gather -- input x = (F / h, G / h^2), output t = (U, h P) -- the exact local
// solve t = M x has the same matrix M on every level:
//   M = [[h Kuu, h^2 Kup], [h^2 Kpu, h^3 Kpp]],  K_j^+ = [[Kuu, Kup], [Kpu, Kpp]].
// K_j^+ is formed through the Schur complement of Sec. 3.2 (with the
// pseudo-inverse S^+ on mean-zero pressures, which equals the pseudo-inverse
// of K_j, Sec. 3.3):
//   Kuu = A^-1 - A^-1 B^T S^+ B A^-1,  Kup = A^-1 B^T S^+,  Kpu = Kup^T,  Kpp = -S^+,
// with A^-1 dense from the fast diagonalization (Eqs. inverse2d /
// fast_inverse extended to 3D) and S^+ = (S + a 1 1^T)^-1 - 1 1^T / (a NP^2)
// (S is positive definite on mean-zero vectors and S 1 = 0).  Everything in
// FP64 on the host; M is built from two levels and the two must agree.
#include "direct.hpp"

#include <cmath>
#include <stdexcept>

#include "tables.hpp"

namespace smg {

namespace {

// A^-1 of velocity component c (dense, NV x NV) from the interior-type FD
// tables: (S2 x S1 x S0) diag(1 / (l0 + l1 + l2)) (S2 x S1 x S0)^T
std::vector<double> fd_inverse_dense(const std::vector<double>& t, int k, int c) {
    const int nc = 2 * k + 1, nd = 2 * k + 2;
    const int oSC = 0, oLC = nc * nc, oSD = oLC + nc, oLD = oSD + 4 * nd * nd;
    int ext[3];
    const double* S[3];
    const double* L[3];
    for (int d = 0; d < 3; ++d) {
        ext[d] = d == c ? nc : nd;
        S[d] = d == c ? &t[oSC] : &t[oSD];      // boundary type 0: interior window
        L[d] = d == c ? &t[oLC] : &t[oLD];
    }
    const int nv = ext[0] * ext[1] * ext[2];
    // Q[e][mode] = S0[i0][m0] S1[i1][m1] S2[i2][m2]
    std::vector<double> Q(size_t(nv) * nv), lam(nv);
    for (int m2 = 0; m2 < ext[2]; ++m2)
        for (int m1 = 0; m1 < ext[1]; ++m1)
            for (int m0 = 0; m0 < ext[0]; ++m0) {
                const int md = m0 + ext[0] * (m1 + ext[1] * m2);
                lam[md] = L[0][m0] + L[1][m1] + L[2][m2];
                for (int i2 = 0; i2 < ext[2]; ++i2)
                    for (int i1 = 0; i1 < ext[1]; ++i1)
                        for (int i0 = 0; i0 < ext[0]; ++i0) {
                            const int e = i0 + ext[0] * (i1 + ext[1] * i2);
                            Q[size_t(e) * nv + md] =
                                S[0][i0 * ext[0] + m0] * S[1][i1 * ext[1] + m1] * S[2][i2 * ext[2] + m2];
                        }
            }
    std::vector<double> Ainv(size_t(nv) * nv, 0.0), QD(size_t(nv) * nv);
    for (int e = 0; e < nv; ++e)
        for (int md = 0; md < nv; ++md) QD[size_t(e) * nv + md] = Q[size_t(e) * nv + md] / lam[md];
    for (int e = 0; e < nv; ++e)
        for (int f = 0; f < nv; ++f) {
            double s = 0.0;
            const double* a = &QD[size_t(e) * nv];
            const double* b = &Q[size_t(f) * nv];
            for (int md = 0; md < nv; ++md) s += a[md] * b[md];
            Ainv[size_t(e) * nv + f] = s;
        }
    return Ainv;
}

// dense B (NP x 3 NV): (B u)_p = - sum_c prod_{d != c} md[i_d] sum_j D[i_c][j] u_c(...)
std::vector<double> divergence_dense(const std::vector<double>& t, int k) {
    const int nc = 2 * k + 1, nd = 2 * k + 2;
    const int oDP = nc * nc + nc + 4 * nd * nd + 4 * nd, oMD = oDP + nd * nc;
    const int nv = nc * nd * nd, np = nd * nd * nd;
    std::vector<double> B(size_t(np) * 3 * nv, 0.0);
    for (int p = 0; p < np; ++p) {
        const int q[3] = {p % nd, (p / nd) % nd, p / (nd * nd)};
        for (int c = 0; c < 3; ++c) {
            int ext[3];
            for (int d = 0; d < 3; ++d) ext[d] = d == c ? nc : nd;
            double mass = 1.0;
            for (int d = 0; d < 3; ++d)
                if (d != c) mass *= t[oMD + q[d]];
            for (int j = 0; j < nc; ++j) {
                int i[3] = {q[0], q[1], q[2]};
                i[c] = j;
                const int e = i[0] + ext[0] * (i[1] + ext[1] * i[2]);
                B[size_t(p) * 3 * nv + c * nv + e] -= mass * t[oDP + q[c] * nc + j];
            }
        }
    }
    return B;
}

// inverse of a symmetric positive definite matrix (Cholesky, in place)
void spd_inverse(std::vector<double>& A, int n) {
    std::vector<double> L(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[size_t(j) * n + j];
        for (int q = 0; q < j; ++q) d -= L[size_t(j) * n + q] * L[size_t(j) * n + q];
        if (!(d > 0.0)) throw std::runtime_error("direct solver: Schur complement not positive definite");
        const double ljj = std::sqrt(d);
        L[size_t(j) * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[size_t(i) * n + j];
            for (int q = 0; q < j; ++q) s -= L[size_t(i) * n + q] * L[size_t(j) * n + q];
            L[size_t(i) * n + j] = s / ljj;
        }
    }
    // inverse of L (lower triangular), then A^-1 = L^-T L^-1
    std::vector<double> Li(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        Li[size_t(j) * n + j] = 1.0 / L[size_t(j) * n + j];
        for (int i = j + 1; i < n; ++i) {
            double s = 0.0;
            for (int q = j; q < i; ++q) s -= L[size_t(i) * n + q] * Li[size_t(q) * n + j];
            Li[size_t(i) * n + j] = s / L[size_t(i) * n + i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int q = i; q < n; ++q) s += Li[size_t(q) * n + i] * Li[size_t(q) * n + j];
            A[size_t(i) * n + j] = A[size_t(j) * n + i] = s;
        }
}

// M (d x d, row-major [out][in]) from the patch tables of a level with cell size h
std::vector<double> normalized_map(const std::vector<double>& t, int k, double h) {
    const int nc = 2 * k + 1, nd = 2 * k + 2;
    const int nv = nc * nd * nd, nu = 3 * nv, np = nd * nd * nd, d = nu + np;
    std::vector<double> Ai[3];
    for (int c = 0; c < 3; ++c) Ai[c] = fd_inverse_dense(t, k, c);
    const std::vector<double> B = divergence_dense(t, k);
    // W = A^-1 B^T (nu x np), block diagonal A
    std::vector<double> W(size_t(nu) * np, 0.0);
    for (int c = 0; c < 3; ++c)
        for (int e = 0; e < nv; ++e)
            for (int p = 0; p < np; ++p) {
                double s = 0.0;
                for (int f = 0; f < nv; ++f) s += Ai[c][size_t(e) * nv + f] * B[size_t(p) * nu + c * nv + f];
                W[size_t(c * nv + e) * np + p] = s;
            }
    // S = B W (np x np), then S^+
    std::vector<double> Sp(size_t(np) * np, 0.0);
    double tr = 0.0;
    for (int p = 0; p < np; ++p)
        for (int q = 0; q < np; ++q) {
            double s = 0.0;
            for (int u = 0; u < nu; ++u) s += B[size_t(p) * nu + u] * W[size_t(u) * np + q];
            Sp[size_t(p) * np + q] = s;
        }
    for (int p = 0; p < np; ++p) tr += Sp[size_t(p) * np + p];
    const double a = tr / np / np;
    for (auto& v : Sp) v += a;
    spd_inverse(Sp, np);
    const double corr = 1.0 / (a * double(np) * np);
    for (auto& v : Sp) v -= corr;
    // WS = W S^+ (nu x np)
    std::vector<double> WS(size_t(nu) * np, 0.0);
    for (int u = 0; u < nu; ++u)
        for (int q = 0; q < np; ++q) {
            double s = 0.0;
            for (int p = 0; p < np; ++p) s += W[size_t(u) * np + p] * Sp[size_t(p) * np + q];
            WS[size_t(u) * np + q] = s;
        }
    std::vector<double> M(size_t(d) * d, 0.0);
    const double h2 = h * h, h3 = h2 * h;
    for (int u = 0; u < nu; ++u) {
        const int c = u / nv, e = u - c * nv;
        for (int v = 0; v < nu; ++v) {
            double s = (v / nv == c) ? Ai[c][size_t(e) * nv + (v - c * nv)] : 0.0;
            for (int p = 0; p < np; ++p) s -= WS[size_t(u) * np + p] * W[size_t(v) * np + p];
            M[size_t(u) * d + v] = h * s;                                        // h Kuu
        }
        for (int q = 0; q < np; ++q) {
            M[size_t(u) * d + nu + q] = h2 * WS[size_t(u) * np + q];            // h^2 Kup
            M[size_t(nu + q) * d + u] = h2 * WS[size_t(u) * np + q];            // h^2 Kpu
        }
    }
    for (int p = 0; p < np; ++p)
        for (int q = 0; q < np; ++q) M[size_t(nu + p) * d + nu + q] = -h3 * Sp[size_t(p) * np + q];   // h^3 Kpp
    return M;
}

}  // namespace

std::vector<double> direct_interior_map(const Ref1D& r, double penalty_factor) {
    const int k = r.k;
    const std::vector<double> M4 = normalized_map(build_patch_tables(r, 4, penalty_factor), k, 0.25);
    const std::vector<double> M8 = normalized_map(build_patch_tables(r, 8, penalty_factor), k, 0.125);
    double scale = 0.0, err = 0.0;
    for (size_t i = 0; i < M4.size(); ++i) {
        scale = std::fmax(scale, std::fabs(M4[i]));
        err = std::fmax(err, std::fabs(M4[i] - M8[i]));
    }
    if (!(err <= 1e-9 * scale))
        throw std::runtime_error("direct solver: the normalized interior map differs between levels");
    return M4;
}

}  // namespace smg
