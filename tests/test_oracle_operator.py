"""Pins of the oracle's global operator K = [[A, B^T], [B, 0]] (CPU).

Each test checks the oracle against something other than itself: symmetry
and definiteness that the bilinear form implies, the separable (Kronecker)
route of kron1d, the kernel and rank of B that H(div)-conformity and
div V_h = Q_h imply, exact reproduction of a polynomial solution, and the
O(h^{k+1}) convergence of the L2 errors (Sec. 3.3, Fig. convergence3d).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import manufactured as mf
from kron1d import global_operator
from oracle.stokes import Stokes


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (2, 2), (3, 3), (4, 1), (2, 5)])
def test_symmetric(n, k):
    K = Stokes(n, k).assemble()
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()


@pytest.mark.parametrize("n,k", [(2, 1), (2, 2), (3, 2), (4, 1)])
def test_velocity_block_spd_and_indefinite_k(n, k):
    S = Stokes(n, k)
    K = S.assemble().toarray()
    A = K[:3 * S.nc, :3 * S.nc]
    lam = np.linalg.eigvalsh(A)
    assert lam.min() > 1e-6 * lam.max()
    lamK = np.linalg.eigvalsh(K)
    # saddle point: npres - 1 negative eigenvalues, one zero (constant pressure)
    assert (lamK < -1e-10 * lamK.max()).sum() == S.npres - 1
    assert (np.abs(lamK) < 1e-10 * lamK.max()).sum() == 1


def test_velocity_block_cholesky_n6():
    S = Stokes(6, 1)
    A = S.assemble()[:3 * S.nc, :3 * S.nc].toarray()
    sla.cholesky(A)      # raises if A is not positive definite


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (2, 2), (3, 2), (4, 1), (2, 3), (2, 5)])
def test_kronecker_identity(n, k):
    """3D quadrature assembly == 1D assembly combined by Kronecker products."""
    K = Stokes(n, k).assemble()
    Kk = global_operator(n, k)
    assert abs(K - Kk).max() <= 1e-13 * abs(K).max()


@pytest.mark.parametrize("n,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_divergence_block_kernel_and_rank(n, k):
    S = Stokes(n, k)
    K = S.assemble()
    B = K[3 * S.nc:, :3 * S.nc].toarray()
    # B^T 1 = 0: (1, div v) = 0 for v.n = 0 on the boundary
    assert np.abs(B.T @ np.ones(S.npres)).max() < 1e-13 * np.abs(B).max()
    # div V_h = Q_h cap L2_0: rank B = dim Q_h - 1
    assert np.linalg.matrix_rank(B, tol=1e-10 * np.abs(B).max()) == S.npres - 1


@pytest.mark.parametrize("n,k", [(2, 1), (3, 2), (4, 1)])
def test_divergence_identity(n, k):
    """For the divergence-free polynomial of ``manufactured.poly`` the
    interpolant satisfies B u = 0 exactly (pointwise divergence zero)."""
    S = Stokes(n, k)
    K = S.assemble()
    x = S.interpolate(mf.poly_u, mf.poly_p)
    Bu = K[3 * S.nc:, :3 * S.nc] @ x[:3 * S.nc]
    assert np.abs(Bu).max() <= 1e-12


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (2, 2), (3, 3), (4, 1), (2, 4)])
def test_polynomial_reproduction(n, k):
    """K I_h(u, p) = b exactly for the polynomial solution, and the solve
    returns the interpolant."""
    S = Stokes(n, k)
    K = S.assemble()
    b = S.rhs(mf.poly_f, mf.poly_u)
    xi = S.interpolate(mf.poly_u, mf.poly_p)
    assert np.abs(K @ xi - b).max() <= 1e-12 * np.abs(b).max()
    xs = S.direct_solve(b, K)
    assert np.abs(xs - xi).max() <= 1e-11
    eu, ep = S.l2_errors(xs, mf.poly_u, mf.poly_p)
    assert eu < 1e-12 and ep < 1e-11


@pytest.mark.parametrize("n,k", [(2, 2), (3, 3)])
def test_pressure_only_reproduction(n, k):
    S = Stokes(n, k)
    K = S.assemble()
    b = S.rhs(mf.ponly_f, mf.ponly_u)
    xi = S.interpolate(mf.ponly_u, mf.ponly_p)
    xi = S.normalize_pressure(xi)
    assert np.abs(K @ xi - b).max() <= 1e-12 * np.abs(b).max()
    assert np.abs(S.direct_solve(b, K) - xi).max() <= 1e-11


def test_mismatch_is_detected():
    """The reproduction pin fails when a term is dropped: a penalty factor
    of 1 instead of 2 changes K but not the interpolant."""
    S = Stokes(2, 1, penalty_factor=2.0)
    S2 = Stokes(2, 1, penalty_factor=1.0)
    xi = S.interpolate(mf.poly_u, mf.poly_p)
    b = S.rhs(mf.poly_f, mf.poly_u)
    assert np.abs(S2.assemble() @ xi - b).max() > 1e-3


@pytest.mark.parametrize("k,ns", [(1, (4, 8)), (2, (2, 4)), (2, (4, 8)), (3, (2, 4))])
def test_convergence_order(k, ns):
    errs = []
    for n in ns:
        S = Stokes(n, k)
        x = S.direct_solve(S.rhs(mf.sine_f, mf.sine_u))
        errs.append(S.l2_errors(x, mf.sine_u, mf.sine_p))
    rate_u = np.log2(errs[0][0] / errs[1][0])
    rate_p = np.log2(errs[0][1] / errs[1][1])
    assert rate_u > k + 1 - 0.25, rate_u
    assert rate_p > k + 1 - 0.25, rate_p


@pytest.mark.parametrize("n,k", [(3, 1), (2, 3)])
def test_matrix_free_and_rows_agree_with_assembly(n, k):
    S = Stokes(n, k)
    K = S.assemble()
    x = np.random.default_rng(7).uniform(-1, 1, S.ndof)
    y = K @ x
    assert np.abs(S.apply(x) - y).max() <= 1e-13 * np.abs(y).max()
    rows = np.array([0, 3, S.nc + 1, 2 * S.nc + 5, S.ndof - 1])
    assert np.abs(S.apply_rows(x, rows) - y[rows]).max() <= 1e-13 * np.abs(y).max()


def test_sizes_table():
    """Unknown counts 3(N1-1)N1^2 + N1^3 (boundary normals eliminated)."""
    expect = {(1, 1): 20, (1, 2): 81, (1, 3): 208, (2, 1): 208, (2, 2): 756, (4, 1): 1856, (4, 2): 6480,
              (16, 2): 435456, (32, 2): 3511296, (64, 1): 8339456, (64, 2): 28200960, (64, 5): 226050048}
    for (n, k), nd in expect.items():
        assert Stokes(n, k).ndof == nd
