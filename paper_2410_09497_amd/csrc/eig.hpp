// Small dense symmetric eigen solvers (host, FP64) for the fast
// diagonalization of the patch matrices (Eqs. inverse2d / fast_inverse).
#pragma once

#include <cmath>
#include <stdexcept>
#include <vector>

#include "fe1d.hpp"

namespace smg {

// Cyclic Jacobi rotations: A = Q diag(lam) Q^T for symmetric A (n small).
inline void jacobi_eig(Dense A, std::vector<double>& lam, Dense& Q) {
    const int n = A.rows;
    Q = Dense(n, n);
    for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A(i, j) * A(i, j);
                if (i != j) off += A(i, j) * A(i, j);
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {          // A <- A J (columns p, q)
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          // A <- J^T A (rows p, q)
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q(k, p), qkq = Q(k, q);
                    Q(k, p) = c * qkp - s * qkq;
                    Q(k, q) = s * qkp + c * qkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A(i, i);
}

// Generalized problem L S = M S Lambda with M SPD: Cholesky M = R R^T,
// C = R^{-1} L R^{-T} = Q Lambda Q^T, S = R^{-T} Q, so S^T M S = I and
// S^T L S = Lambda.
inline void generalized_eig(const Dense& L, const Dense& M, std::vector<double>& lam, Dense& S) {
    const int n = L.rows;
    Dense R(n, n);
    for (int j = 0; j < n; ++j) {
        double d = M(j, j);
        for (int k = 0; k < j; ++k) d -= R(j, k) * R(j, k);
        if (!(d > 0)) throw std::runtime_error("mass matrix not positive definite");
        R(j, j) = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = M(i, j);
            for (int k = 0; k < j; ++k) v -= R(i, k) * R(j, k);
            R(i, j) = v / R(j, j);
        }
    }
    // X = R^{-1} L (forward substitution on columns), C = X R^{-T}
    Dense X(n, n), C(n, n);
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double v = L(i, c);
            for (int k = 0; k < i; ++k) v -= R(i, k) * X(k, c);
            X(i, c) = v / R(i, i);
        }
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i) {
            double v = X(r, i);
            for (int k = 0; k < i; ++k) v -= R(i, k) * C(r, k);
            C(r, i) = v / R(i, i);
        }
    for (int i = 0; i < n; ++i)       // symmetrize rounding
        for (int j = i + 1; j < n; ++j) C(i, j) = C(j, i) = 0.5 * (C(i, j) + C(j, i));
    Dense Q;
    jacobi_eig(C, lam, Q);
    // S = R^{-T} Q (back substitution)
    S = Dense(n, n);
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double v = Q(i, c);
            for (int k = i + 1; k < n; ++k) v -= R(k, i) * S(k, c);
            S(i, c) = v / R(i, i);
        }
}

}  // namespace smg
