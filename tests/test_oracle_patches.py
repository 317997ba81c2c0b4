"""Pins of the oracle's vertex patches and local solvers (CPU).

* patch counts, colours and DoF sets (Sec. 3.1, Fig. patch_coloring);
* the patch matrix A_j is the Kronecker sum of restricted 1D matrices
  (Sec. 3.2), checked against the independent 1D route of kron1d;
* fast diagonalization (Eqs. inverse2d / fast_inverse, extended to 3D)
  equals the dense inverse of A_j on every patch type;
* the Schur-complement solve of Sec. 3.2 equals the pseudo-inverse ("Direct
  solver" of Sec. 3.3).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from kron1d import patch_1d, kron3
from oracle.stokes import Stokes
from oracle.patches import Patches, schur_local_solve


@pytest.mark.parametrize("n,k", [(2, 1), (3, 1), (4, 2)])
def test_patch_counts_colours_and_cover(n, k):
    S = Stokes(n, k)
    P = Patches(S)
    assert len(P.verts) == (n - 1) ** 3
    assert P.size == 3 * (2 * k + 1) * (2 * k + 2) ** 2 + 8 * (k + 1) ** 3
    seen = np.zeros(S.ndof, dtype=int)
    for c in range(8):
        owner = np.zeros(S.ndof, dtype=int)
        for v in P.verts[P.colour == c]:
            idx = P.dofs(v)
            assert len(idx) == P.size and len(np.unique(idx)) == P.size
            owner[idx] += 1
            seen[idx] += 1
        assert owner.max() <= 1, "patches of one colour overlap"
    assert seen.min() >= 1, "some unknown is in no patch"


def test_single_patch_is_everything():
    S = Stokes(2, 2)
    P = Patches(S)
    assert len(P.verts) == 1
    assert np.array_equal(np.sort(P.dofs(P.verts[0])), np.arange(S.ndof))


def test_patch_dofs_are_supported_in_patch():
    """Every function of X_j vanishes outside the 8 cells: its row of K only
    couples to DoFs of cells that touch the patch (domain of dependence)."""
    S = Stokes(4, 1)
    K = S.assemble().tocsr()
    P = Patches(S)
    v = np.array([2, 2, 2])
    # cells of the patch: {1,2}^3; the pressure DoFs of far cells must not couple
    far = S.pres_global(np.array([[0, 0, 0], [3, 3, 3], [0, 3, 0]])).ravel()
    rows = K[P.dofs(v)][:, far]
    assert rows.nnz == 0 or np.abs(rows.data).max() == 0


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_patch_matrix_is_kronecker_sum_and_fd_inverts_it(k):
    n = 4 if k <= 3 else 3
    S = Stokes(n, k)
    K = S.assemble()
    P = Patches(S)
    nv = P.nvel
    for v in ([1, 1, 1], [2, 1, n - 1], [n - 1, n - 1, 2]):
        v = np.array(v)
        Kj = P.local_matrix(K, v)
        one = [patch_1d(n, k, v[d]) for d in range(3)]
        for c in range(3):
            # Kronecker sum of the restricted 1D matrices (x fastest)
            facs = []
            for d in range(3):
                if d == c:
                    facs.append((one[d]["Lc"], one[d]["Mc"]))
                else:
                    facs.append((one[d]["Ld"], one[d]["Md"]))
            (Lx, Mx), (Ly, My), (Lz, Mz) = facs
            Akr = (kron3(Mz, My, Lx) + kron3(Mz, Ly, Mx) + kron3(Lz, My, Mx)).toarray()
            Ac = Kj[c * nv:(c + 1) * nv, c * nv:(c + 1) * nv]
            assert np.abs(Ac - Akr).max() <= 1e-12 * np.abs(Ac).max()
            # fast diagonalization: L S = M S Lambda, S^T M S = I
            ev = []
            for (L, M) in facs:
                lam, Sv = sla.eigh(L, M)
                assert np.abs(Sv.T @ M @ Sv - np.eye(len(lam))).max() < 1e-10
                assert np.abs(Sv.T @ L @ Sv - np.diag(lam)).max() < 1e-8 * np.abs(lam).max()
                ev.append((lam, Sv))
            (lx, Sx), (ly, Sy), (lz, Sz) = ev
            Sall = np.kron(Sz, np.kron(Sy, Sx))
            lam3 = (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]).ravel()
            Ainv_fd = (Sall / lam3) @ Sall.T
            Ainv = np.linalg.inv(Ac)
            assert np.abs(Ainv_fd - Ainv).max() <= 1e-10 * np.abs(Ainv).max()


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (3, 3)])
def test_schur_equals_pseudo_inverse(n, k):
    S = Stokes(n, k)
    K = S.assemble()
    P = Patches(S)
    rng = np.random.default_rng(11)
    for v in P.verts[:: max(1, len(P.verts) // 3)]:
        Kj = P.local_matrix(K, v)
        Kp = P.pinv(K, v)
        assert np.abs(Kj @ Kp @ Kj - Kj).max() <= 1e-10 * np.abs(Kj).max()
        r = rng.uniform(-1, 1, P.size)
        a = P.local_solve(K, v, r)
        b = schur_local_solve(Kj, 3 * P.nvel, r)
        assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()


def test_patch_pressure_kernel():
    """Constant patch pressure is the only kernel of K_j (B_j^T 1 = 0 because
    v.n = 0 on the patch boundary for every v in X_j)."""
    S = Stokes(4, 1)
    P = Patches(S)
    Kj = P.local_matrix(S.assemble(), np.array([2, 2, 2]))
    z = np.zeros(P.size)
    z[3 * P.nvel:] = 1.0
    assert np.abs(Kj @ z).max() < 1e-13
    lam = np.linalg.eigvalsh(Kj)
    assert (np.abs(lam) < 1e-10 * np.abs(lam).max()).sum() == 1


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (3, 3)])
def test_bordered_route_equals_pseudo_inverse(n, k):
    """The bordered sparse-LU route to K_j^+ r (used for degrees 4, 5) equals
    the dense pseudo-inverse on every patch type, also for a right-hand side
    whose patch pressure part has nonzero mean.  Both are exact up to
    rounding: at k = 3 the eigendecomposition route leaves a relative
    residual ||K_j x - r'|| of about 5e-11 (the bordered LU 2e-12), which the
    saddle-point system turns into differences of about 1e-10 relative, so
    the bound is 1e-9."""
    S = Stokes(n, k)
    K = S.assemble()
    Pd, Pb = Patches(S), Patches(S, solver="bordered")
    rng = np.random.default_rng(5)
    for v in Pd.verts:
        r = rng.uniform(-1, 1, Pd.size)
        a = Pd.local_solve(K, v, r)
        b = Pb.local_solve(K, v, r)
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()


@pytest.mark.parametrize("k", [4, 5])
def test_bordered_route_solves_large_patches(k):
    """Degrees 4, 5 (one patch on 2^3 cells): K_j x = r - mean-part and
    x has zero patch-pressure mean, i.e. x = K_j^+ r."""
    S = Stokes(2, k)
    K = S.assemble()
    P = Patches(S, solver="bordered")
    v = P.verts[0]
    Kj = P.local_matrix(K, v)
    r = np.random.default_rng(k).uniform(-1, 1, P.size)
    x = P.local_solve(K, v, r)
    c = np.zeros(P.size)
    c[3 * P.nvel:] = 1.0
    rp = r - (c @ r) / (c @ c) * c
    assert abs(c @ x) <= 1e-10 * np.abs(x).max()
    assert np.abs(Kj @ x - rp).max() <= 1e-9 * np.abs(rp).max()
