"""The 2D workload of Table 1 (exact-2d) on the oracle (CPU): the method of
Secs. 2-3 in two dimensions with the pseudo-inverse ("Direct") local solver,
GMRES to 1e-8 preconditioned by the V-cycle, right-hand side of Sec. 3.3.
The paper does not give mu and sigma of its phi; they are read as 1/2 and
1/4.  The table's labels Q_3 .. Q_8 are read as the pair RT_k / DG Q_k with
k = 3 .. 8 and L as 2^L cells per direction (tests/golden/table_exact2d.json).
The printed values are met with two smoothing sweeps before and after the
coarse correction; with one they are not.

Pins of the 2D operator itself: symmetry and the O(h^{k+1}) velocity error of
the manufactured solution, which also checks f = -Laplace(u) + grad(p)."""
import json
import os

import numpy as np
import pytest

from oracle.mg import fgmres, fractional_iterations
from oracle.stokes2d import Multigrid2D, Stokes2D, manufactured_2d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table_exact2d.json")
U, P, F, PHI = manufactured_2d(0.5, 0.25)


def _solve(n, k, rtol, sweeps=1):
    mg = Multigrid2D(n, k)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(F)
    x, hist = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v, pre=sweeps, post=sweeps), rtol=rtol, restart=50)
    return S, K, b, x, hist


def test_phi_derivatives_by_differences():
    """The closed-form derivatives of phi against central differences."""
    x = np.linspace(0.05, 0.95, 19)
    h = 1e-5
    for m in (1, 2, 3):
        fd = (PHI(x + h, m - 1) - PHI(x - h, m - 1)) / (2 * h)
        assert np.abs(fd - PHI(x, m)).max() <= 1e-5 * (1 + np.abs(PHI(x, m)).max()), m
    # phi and phi' vanish at both ends: u = 0 on the boundary
    for m in (0, 1):
        assert abs(PHI(np.array([0.0, 1.0]), m)).max() <= 1e-15


def test_operator_symmetric_and_pressure_kernel():
    S = Stokes2D(4, 2)
    K = S.assemble()
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    c = np.zeros(S.ndof)
    c[S.offsets[2]:] = 1.0                       # constant pressure
    assert np.abs(K @ c).max() <= 1e-10 * abs(K).max()


@pytest.mark.parametrize("k,ns", [(1, (8, 16)), (2, (8, 16))])
def test_velocity_error_order(k, ns):
    errs = []
    for n in ns:
        S, K, b, x, hist = _solve(n, k, 1e-11)
        assert hist[-1] <= 1e-11
        errs.append(S.l2_velocity_error(x, U))
    rate = np.log2(errs[0] / errs[1])
    assert rate > k + 1 - 0.25, rate


def _nu(n, k, sweeps=1):
    _, _, _, _, hist = _solve(n, k, 1e-8, sweeps)
    return fractional_iterations(hist)


def test_table_exact2d_trends():
    """Table 1's two observations (Sec. 3.3): the iteration count does not
    grow with the level, and it falls with the degree.  Measured at L = 3, 4
    (k = 3 .. 7): 3.81 / 4.07, 2.97 / 2.99, 2.55 / 2.74, 2.44 / 2.56,
    2.26 / 2.37; from k = 4 on one level more adds at most 0.25, and nu falls
    with the degree at both levels."""
    nu = {(L, k): _nu(2 ** L, k) for L in (3, 4) for k in range(3, 8)}
    for k in range(4, 8):
        assert nu[(4, k)] - nu[(3, k)] <= 0.25, (k, nu[(3, k)], nu[(4, k)])
    for L in (3, 4):
        seq = [nu[(L, k)] for k in range(3, 8)]
        assert all(a > b for a, b in zip(seq, seq[1:])), (L, seq)


@pytest.mark.xfail(strict=True, reason="with the single pre- and post-smoothing sweep the paper's text states, nu at "
                                       "L = 3, 4 is 0.24 .. 1.0 above Table 1's Direct column (k = 3: 3.81 / 4.07 "
                                       "against 2.8 / 3.2; k = 7: 2.26 / 2.37 against 1.9 / 2.1); two sweeps match it "
                                       "(test_table_exact2d_direct_values_two_sweeps)")
def test_table_exact2d_direct_values():
    gold = json.load(open(GOLDEN))
    for L in (3, 4):
        for j, k in enumerate(gold["degrees"][:5]):
            paper = gold["direct"][str(L)][j]
            assert abs(_nu(2 ** L, k) - paper) <= 0.3, (L, k, paper)


def test_table_exact2d_direct_values_two_sweeps():
    """Table 1's Direct column is met when the V-cycle smooths twice before
    and twice after the coarse correction: nu within 0.25 of the printed
    value at L = 3 for Q_3 .. Q_8 and at L = 4 for Q_3 .. Q_6 (measured
    differences at most 0.22: L = 3: 2.99 2.30 2.13 1.99 1.88 1.88 against
    2.8 2.4 2.1 2.2 1.9 2.1; L = 4: 3.19 2.42 2.26 2.07 against 3.2 2.4 2.3
    2.2).  The same two sweeps give the 3D claims of Sec. 3.3 and Table
    vs_poisson on the GPU (tests/test_gpu_solver.py)."""
    gold = json.load(open(GOLDEN))
    for L, nk in ((3, 6), (4, 4)):
        for j, k in enumerate(gold["degrees"][:nk]):
            paper = gold["direct"][str(L)][j]
            nu = _nu(2 ** L, k, sweeps=2)
            assert abs(nu - paper) <= 0.25, (L, k, nu, paper)
