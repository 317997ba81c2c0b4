// The "Direct" local solver of Sec. 3.3 (the pseudo-inverse of the patch
// matrix), as one dense matrix per patch type.
//
// A vertex patch (8 cells around vertex v) has the patch matrix
// K_j(h) = [[h A^, h^2 B^T], [h^2 B^, 0]] with A^, B^ independent of the level:
// A_j scales like h (the interior penalty 2 (k+1)^2 / h included, on interior
// and boundary faces alike), B_j like h^2.  A^ depends on the patch only
// through which outer faces lie on the domain boundary, per direction (the
// four 1D window types of the fast diagonalization); B^ is the same for all.
// In the normalized variables of the patch gather -- input x = (F / h, G / h^2),
// output t = (U, h P) -- the exact local solve t = M x therefore has one
// matrix per type on every level:
//   M = [[h Kuu, h^2 Kup], [h^2 Kpu, h^3 Kpp]],  K_j^+ = [[Kuu, Kup], [Kpu, Kpp]].
// K_j^+ is formed through the Schur complement of Sec. 3.2 (with the
// pseudo-inverse S^+ on mean-zero pressures, which equals the pseudo-inverse
// of K_j, Sec. 3.3):
//   Kuu = A^-1 - A^-1 B^T S^+ B A^-1,  Kup = A^-1 B^T S^+,  Kpu = Kup^T,  Kpp = -S^+,
// with A^-1 dense from the fast diagonalization (Eqs. inverse2d /
// fast_inverse extended to 3D) and S^+ = (S + a 1 1^T)^-1 - 1 1^T / (a NP^2)
// (S is positive definite on mean-zero vectors and S 1 = 0).  Everything in
// FP64 on the host; every M is built from two levels and the two must agree.
#include "direct.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <mutex>
#include <stdexcept>
#include <thread>

#include "tables.hpp"

namespace smg {

namespace {

// C (m x n) = A (m x q) B (q x n), all row-major; the inner loop runs over
// contiguous columns of B and C
void matmul(const double* A, const double* B, double* C, int m, int q, int n) {
    std::fill(C, C + size_t(m) * n, 0.0);
    for (int i = 0; i < m; ++i) {
        double* c = C + size_t(i) * n;
        for (int p = 0; p < q; ++p) {
            const double a = A[size_t(i) * q + p];
            if (a == 0.0) continue;
            const double* b = B + size_t(p) * n;
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

std::vector<double> transpose(const std::vector<double>& A, int m, int n) {
    std::vector<double> T(size_t(m) * n);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) T[size_t(j) * m + i] = A[size_t(i) * n + j];
    return T;
}

// A^-1 of velocity component c (dense, NV x NV) from the FD tables, with
// window type ty[d] in the two directions d != c (the continuous window of
// direction c is the same for every patch):
//   (S2 x S1 x S0) diag(1 / (l0 + l1 + l2)) (S2 x S1 x S0)^T
std::vector<double> fd_inverse_dense(const std::vector<double>& t, int k, int c, const int ty[3]) {
    const int nc = 2 * k + 1, nd = 2 * k + 2;
    const int oSC = 0, oLC = nc * nc, oSD = oLC + nc, oLD = oSD + 4 * nd * nd;
    int ext[3];
    const double* S[3];
    const double* L[3];
    for (int d = 0; d < 3; ++d) {
        ext[d] = d == c ? nc : nd;
        S[d] = d == c ? &t[oSC] : &t[oSD + ty[d] * nd * nd];
        L[d] = d == c ? &t[oLC] : &t[oLD + ty[d] * nd];
    }
    const int nv = ext[0] * ext[1] * ext[2];
    // Q[e][mode] = S0[i0][m0] S1[i1][m1] S2[i2][m2]
    std::vector<double> Q(size_t(nv) * nv), QD(size_t(nv) * nv);
    for (int m2 = 0; m2 < ext[2]; ++m2)
        for (int m1 = 0; m1 < ext[1]; ++m1)
            for (int m0 = 0; m0 < ext[0]; ++m0) {
                const int md = m0 + ext[0] * (m1 + ext[1] * m2);
                const double lam = L[0][m0] + L[1][m1] + L[2][m2];
                for (int i2 = 0; i2 < ext[2]; ++i2)
                    for (int i1 = 0; i1 < ext[1]; ++i1)
                        for (int i0 = 0; i0 < ext[0]; ++i0) {
                            const int e = i0 + ext[0] * (i1 + ext[1] * i2);
                            const double q = S[0][i0 * ext[0] + m0] * S[1][i1 * ext[1] + m1] * S[2][i2 * ext[2] + m2];
                            Q[size_t(e) * nv + md] = q;
                            QD[size_t(e) * nv + md] = q / lam;
                        }
            }
    std::vector<double> Ainv(size_t(nv) * nv);
    matmul(QD.data(), transpose(Q, nv, nv).data(), Ainv.data(), nv, nv, nv);
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

// M (d x d, row-major [out][in]) of window types ty from the patch tables of a level with cell size h
std::vector<double> normalized_map(const std::vector<double>& t, int k, double h, const int ty[3]) {
    const int nc = 2 * k + 1, nd = 2 * k + 2;
    const int nv = nc * nd * nd, nu = 3 * nv, np = nd * nd * nd, d = nu + np;
    std::vector<double> Ai[3];
    for (int c = 0; c < 3; ++c) Ai[c] = fd_inverse_dense(t, k, c, ty);
    const std::vector<double> B = divergence_dense(t, k);
    const std::vector<double> Bt = transpose(B, np, nu);
    // W = A^-1 B^T (nu x np), block diagonal A
    std::vector<double> W(size_t(nu) * np);
    for (int c = 0; c < 3; ++c)
        matmul(Ai[c].data(), Bt.data() + size_t(c) * nv * np, W.data() + size_t(c) * nv * np, nv, nv, np);
    // S = B W (np x np), then S^+
    std::vector<double> Sp(size_t(np) * np);
    matmul(B.data(), W.data(), Sp.data(), np, nu, np);
    double tr = 0.0;
    for (int p = 0; p < np; ++p) tr += Sp[size_t(p) * np + p];
    const double a = tr / np / np;
    for (auto& v : Sp) v += a;
    spd_inverse(Sp, np);
    const double corr = 1.0 / (a * double(np) * np);
    for (auto& v : Sp) v -= corr;
    // WS = W S^+ (nu x np); Kuu = A^-1 - WS W^T
    std::vector<double> WS(size_t(nu) * np), Kuu(size_t(nu) * nu);
    matmul(W.data(), Sp.data(), WS.data(), nu, np, np);
    matmul(WS.data(), transpose(W, nu, np).data(), Kuu.data(), nu, np, nu);
    std::vector<double> M(size_t(d) * d, 0.0);
    const double h2 = h * h, h3 = h2 * h;
    for (int u = 0; u < nu; ++u) {
        const int c = u / nv, e = u - c * nv;
        for (int v = 0; v < nu; ++v) {
            const double ai = (v / nv == c) ? Ai[c][size_t(e) * nv + (v - c * nv)] : 0.0;
            M[size_t(u) * d + v] = h * (ai - Kuu[size_t(u) * nu + v]);            // h Kuu
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

void window_types(int type, int ty[3]) {
    if (type == kDirectTypes - 1) {
        ty[0] = ty[1] = ty[2] = 3;
    } else {
        ty[0] = type % 3;
        ty[1] = (type / 3) % 3;
        ty[2] = type / 9;
    }
}

// the map of one type from two levels' tables, which must agree
std::vector<double> checked_map(const std::vector<double>& t4, const std::vector<double>& t8, int k, int type) {
    int ty[3];
    window_types(type, ty);
    const std::vector<double> M4 = normalized_map(t4, k, 0.25, ty);
    const std::vector<double> M8 = normalized_map(t8, k, 0.125, ty);
    double scale = 0.0, err = 0.0;
    for (size_t i = 0; i < M4.size(); ++i) {
        scale = std::fmax(scale, std::fabs(M4[i]));
        err = std::fmax(err, std::fabs(M4[i] - M8[i]));
    }
    if (!(err <= 1e-9 * scale))
        throw std::runtime_error("direct solver: the normalized patch map differs between levels");
    return M4;
}

}  // namespace

std::vector<double> direct_type_map(const Ref1D& r, double penalty_factor, int type) {
    if (type < 0 || type >= kDirectTypes) throw std::invalid_argument("direct solver: patch type out of range");
    return checked_map(build_patch_tables(r, 4, penalty_factor), build_patch_tables(r, 8, penalty_factor), r.k, type);
}

std::vector<std::vector<double>> direct_type_maps(const Ref1D& r, double penalty_factor) {
    const std::vector<double> t4 = build_patch_tables(r, 4, penalty_factor);
    const std::vector<double> t8 = build_patch_tables(r, 8, penalty_factor);
    std::vector<std::vector<double>> maps(kDirectTypes);
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto work = [&]() {
        for (int ty = next++; ty < kDirectTypes; ty = next++) {
            try {
                maps[ty] = checked_map(t4, t8, r.k, ty);
            } catch (...) {
                std::lock_guard<std::mutex> g(mu);
                if (!err) err = std::current_exception();
            }
        }
    };
    const int nt = int(std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency())));
    std::vector<std::thread> pool;
    for (int i = 1; i < nt; ++i) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    if (err) std::rethrow_exception(err);
    return maps;
}

}  // namespace smg
