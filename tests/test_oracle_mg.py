"""Pins of the oracle's smoother, transfers, V-cycle and FGMRES (CPU)."""
import json
import os

import numpy as np
import pytest

import manufactured as mf
from oracle.stokes import Stokes
from oracle.patches import Patches
from oracle.mg import Multigrid, prolongation, fgmres, fractional_iterations

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_iterations.json")


@pytest.mark.parametrize("k", [1, 2])
def test_one_patch_sweep_is_exact_solve(k):
    """n = 2: the single vertex patch holds every unknown, so one sweep of
    Alg. 2 from x = 0 is the exact (pseudo-inverse) solve."""
    mg = Multigrid(2, k)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    x = mg.smooth(1, np.zeros(S.ndof), b)
    assert np.abs(S.normalize_pressure(x) - S.direct_solve(b, K)).max() <= 1e-10


def test_sweep_equals_brute_force_operator():
    """n = 4, k = 1: the loop of Alg. 2 equals the dense product over colours
    of (I - sum_{j in c} R_j^T K_j^+ R_j K) applied to the error, plus the
    matching affine part."""
    mg = Multigrid(4, 1)
    S, K = mg.fine["S"], mg.fine["K"]
    Pt = mg.fine["patches"]
    Kd = K.toarray()
    N = S.ndof
    rng = np.random.default_rng(3)
    x0 = rng.uniform(-1, 1, N)
    b = rng.uniform(-1, 1, N)
    x = x0.copy()
    for c in range(8):
        C = np.zeros((N, N))
        for v in Pt.verts[Pt.colour == c]:
            idx = Pt.dofs(v)
            C[np.ix_(idx, idx)] += Pt.pinv(K, v)
        x = x + C @ (b - Kd @ x)
    assert np.abs(mg.smooth(2, x0, b) - x).max() <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_prolongation_is_embedding(k):
    """Nestedness: the prolonged coefficients describe the same function."""
    Sc, Sf = Stokes(2, k), Stokes(4, k)
    P = prolongation(Sc, Sf)
    xc = np.random.default_rng(0).uniform(-1, 1, Sc.ndof)
    xf = P @ xc
    pts = np.random.default_rng(1).uniform(0, 1, (40, 3))

    def evaluate(S, x, pt):
        cell = np.minimum((pt / S.h).astype(int), S.n - 1)
        ref = pt / S.h - cell
        xe = np.concatenate([x, [0.0]])
        out = []
        for c in range(3):
            V, _ = S.eval_vel(c, ref[None])
            out.append(xe[S.vel_global(c, cell[None])[0]] @ V[:, 0])
        out.append(x[S.pres_global(cell[None])[0]] @ S.eval_pres(ref[None])[:, 0])
        return np.array(out)

    err = max(np.abs(evaluate(Sc, xc, p) - evaluate(Sf, xf, p)).max() for p in pts)
    assert err <= 1e-13
    # a polynomial of X_H is interpolated to the interpolant of X_h
    xi_c = Sc.interpolate(mf.poly_u, mf.poly_p)
    xi_f = Sf.interpolate(mf.poly_u, mf.poly_p)
    assert np.abs(P @ xi_c - xi_f).max() <= 1e-13


@pytest.mark.parametrize("k", [1, 2])
def test_coarse_pseudo_inverse(k):
    mg = Multigrid(1, k)
    K0 = mg.levels[0]["K"].toarray()
    assert np.abs(K0 @ mg.K0_pinv @ K0 - K0).max() <= 1e-10 * np.abs(K0).max()


def test_two_level_with_exact_top_smoother_is_exact():
    """Levels 1^3 and 2^3: the 2^3 smoother is one exact patch solve, so one
    V-cycle solves the system."""
    mg = Multigrid(2, 1)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    x = mg.vcycle(b)
    assert np.abs(S.normalize_pressure(x) - S.direct_solve(b, K)).max() <= 1e-10


def test_fgmres_identity_preconditioner_matches_minimal_residual():
    """Without a preconditioner GMRES minimizes ||b - K x|| over the Krylov
    space; compare with the least-squares solution over an explicit basis."""
    S = Stokes(2, 1)
    K = S.assemble()
    Kd = K.toarray()
    b = np.random.default_rng(5).uniform(-1, 1, S.ndof)
    b[3 * S.nc:] -= b[3 * S.nc:].mean()
    x, hist = fgmres(lambda v: K @ v, b, lambda v: v, rtol=1e-30, restart=12, maxit=12)
    for m in (1, 4, 8, 12):
        Kr = [b]
        for _ in range(m - 1):
            Kr.append(Kd @ Kr[-1])
        Q, _ = np.linalg.qr(np.array(Kr).T)
        y = np.linalg.lstsq(Kd @ Q, b, rcond=None)[0]
        res = np.linalg.norm(b - Kd @ (Q @ y)) / np.linalg.norm(b)
        assert abs(hist[m] - res) <= 1e-8 * max(res, 1e-12) + 1e-13


def test_fgmres_exact_preconditioner_one_step():
    S = Stokes(2, 1)
    K = S.assemble()
    b = S.rhs(mf.sine_f, mf.sine_u)
    x, hist = fgmres(lambda v: K @ v, b, lambda v: S.direct_solve(v, K), rtol=1e-8)
    assert len(hist) == 2 and hist[-1] < 1e-10


def test_fractional_iterations_formula():
    # exactly 1e-2 per step: four steps reach 1e-8
    assert abs(fractional_iterations([1.0, 1e-2, 1e-4, 1e-6, 1e-8]) - 4.0) < 1e-12
    assert abs(fractional_iterations([1.0, 1e-4, 1e-8, 1e-12]) - 2.0) < 1e-12


def test_mg_fgmres_matches_paper_three_step_claim():
    """Sec. 3.3: from k = 3 on, at most three GMRES steps to 1e-8 in 3D."""
    gold = json.load(open(GOLDEN))["three_d_max_steps_from_k3"]
    mg = Multigrid(4, gold["k_min"])
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    x, hist = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v), rtol=gold["rtol"])
    assert len(hist) - 1 <= gold["max_steps"]
    assert np.linalg.norm(b - K @ x) <= gold["rtol"] * np.linalg.norm(b)


@pytest.mark.parametrize("n,k,max_it", [(4, 1, 8), (8, 1, 11), (4, 2, 5), (8, 2, 6)])
def test_mg_fgmres_iterations_level_robust(n, k, max_it):
    """Iteration counts stay bounded as the mesh is refined (Sec. 3.3)."""
    mg = Multigrid(n, k)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    x, hist = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v), rtol=1e-8)
    assert len(hist) - 1 <= max_it
    r = b - K @ x
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)


def _dense_gmres_history(T, b, steps):
    """Relative residuals min ||b - T y|| / ||b|| over the Krylov spaces
    K_m(T, b), m = 0..steps: Arnoldi with modified Gram-Schmidt twice, then
    the small least-squares problem solved directly at every m."""
    nb = np.linalg.norm(b)
    Q = np.zeros((len(b), steps + 1))
    H = np.zeros((steps + 1, steps))
    Q[:, 0] = b / nb
    hist = [1.0]
    for m in range(steps):
        w = T @ Q[:, m]
        for _ in range(2):
            for i in range(m + 1):
                c = Q[:, i] @ w
                H[i, m] += c
                w = w - c * Q[:, i]
        H[m + 1, m] = np.linalg.norm(w)
        Q[:, m + 1] = w / H[m + 1, m]
        e1 = np.zeros(m + 2)
        e1[0] = nb
        y = np.linalg.lstsq(H[:m + 2, :m + 1], e1, rcond=None)[0]
        hist.append(np.linalg.norm(e1 - H[:m + 2, :m + 1] @ y) / nb)
    return hist


def test_vcycle_spectrum_and_fgmres_steps():
    """The V-cycle as a dense operator at 4^3 cells, k = 1 (Sec. 3; the
    columns of P^-1 are V-cycles of the unit vectors, computed in blocks).
    Pins:
    - T = K P^-1 has exactly one zero eigenvalue (the constant pressure,
      the kernel of K) and every other eigenvalue mu has |1 - mu| <= 0.4
      (measured 0.357): the V-cycle is a contraction on the complement;
    - FGMRES with the V-cycle (a fixed linear preconditioner) takes the
      iterates of right-preconditioned GMRES, so its residual history on
      the sine problem equals that of GMRES on the dense T, computed here
      by an independent Arnoldi process with least squares at every step;
      the step count to 1e-8 it predicts is the oracle's."""
    mg = Multigrid(4, 1)
    S, K = mg.fine["S"], mg.fine["K"]
    N = S.ndof
    Pinv = np.zeros((N, N))
    for j0 in range(0, N, 128):
        m = min(128, N - j0)
        E = np.zeros((N, m))
        E[np.arange(j0, j0 + m), np.arange(m)] = 1.0
        Pinv[:, j0:j0 + m] = mg.vcycle(E)
    # the block V-cycle is the column-wise one
    e = np.zeros(N)
    e[N // 3] = 1.0
    assert np.abs(Pinv[:, N // 3] - mg.vcycle(e)).max() <= 1e-12 * np.abs(Pinv).max()
    T = K @ Pinv
    mu = np.linalg.eigvals(T)
    mu = mu[np.argsort(np.abs(mu))]
    assert abs(mu[0]) <= 1e-10 and abs(mu[1]) >= 0.1
    rho = np.abs(1.0 - mu[1:]).max()
    assert rho <= 0.4, rho
    b = S.rhs(mf.sine_f, mf.sine_u)
    _, hist = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v), rtol=1e-8, restart=30)
    dense = _dense_gmres_history(T, b, len(hist) - 1)
    for j, (a, d) in enumerate(zip(hist, dense)):
        assert abs(a - d) <= 1e-6 * d, (j, a, d)
    predicted = next(m for m, r in enumerate(dense) if r <= 1e-8)
    assert predicted == len(hist) - 1
