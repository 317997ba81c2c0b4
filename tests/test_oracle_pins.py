"""Further pins of the oracle (CPU), each against something other than the
oracle's own formula:

* pressure normalization (L^2_0 of Sec. 2): the integral mean, not the mean
  of the coefficients -- a pressure whose Gauss-point values do not average
  to its integral, and closed-form integrals of polynomials;
* discrete divergence (Sec. 2.1: H(div)-conforming velocities are pointwise
  divergence free): ||B u_h|| of the oracle's direct solution and of its
  multigrid-preconditioned FGMRES solution;
* Adam (Kingma & Ba 2015) beyond the first step: the closed-sum form of the
  moment estimates, and the exact sign step that bias correction gives for a
  constant gradient at every step;
* the learned-solver callbacks: with the exact normalized patch map in place
  of the network, the learned sweep reproduces the exact sweep, and every
  captured pair satisfies t = map(x);
* the contraction monitor of the fallback: synthetic contraction sequences
  trigger at the index where they cross the bound, and a zeroed network
  (correction 0 on interior patches) triggers after the first step.
"""
from fractions import Fraction

import numpy as np
import pytest

import manufactured as mf
from oracle import mlp
from oracle.mg import Multigrid, fgmres
from oracle.stokes import Stokes


# ----------------------------------------------------------------- pressure
def _p_quad(x, y, z):
    return x * x - 1.0 / 3.0 + 0.0 * y + 0.0 * z        # integral over the unit cube: 0


def _f_quad(x, y, z):
    return np.array([2.0 * x, 0.0 * y, 0.0 * z])         # grad p (u = 0)


@pytest.mark.parametrize("n,k", [(2, 2), (3, 2), (2, 3)])
def test_pressure_integral_mean_not_coefficient_mean(n, k):
    """u = 0, p = x^2 - 1/3 (zero integral mean; p in Q_k for k >= 2): the
    discrete solution is (0, I_h p) exactly.  The Gauss-point values of p
    do not average to zero, so a coefficient-mean normalization would shift
    the pressure by a constant and fail."""
    S = Stokes(n, k)
    K = S.assemble()
    b = S.rhs(_f_quad, mf.ponly_u)
    xi = S.interpolate(mf.ponly_u, _p_quad)
    coef_mean = xi[S.offsets[3]:].mean()
    assert abs(coef_mean) > 1e-3                           # the trap is armed
    assert np.abs(K @ xi - b).max() <= 1e-12 * np.abs(b).max()
    assert abs(S.pressure_mean(xi)) <= 1e-14
    xs = S.direct_solve(b, K)
    assert np.abs(xs - xi).max() <= 1e-11


@pytest.mark.parametrize("n,k", [(1, 3), (2, 3), (3, 4)])
def test_pressure_mean_closed_form(n, k):
    """Integral of I_h p over the unit cube for p = x^2 y + z^3 + 2 (in Q_k
    for k >= 3): 1/6 + 1/4 + 2 = 29/12."""
    S = Stokes(n, k)
    xi = S.interpolate(mf.ponly_u, lambda x, y, z: x * x * y + z ** 3 + 2.0)
    assert abs(S.pressure_mean(xi) - 29.0 / 12.0) <= 1e-14
    xn = S.normalize_pressure(xi)
    assert abs(S.pressure_mean(xn)) <= 1e-14
    # normalization shifts the pressure by exactly that constant
    assert np.abs(xi[S.offsets[3]:] - xn[S.offsets[3]:] - 29.0 / 12.0).max() <= 1e-14


# --------------------------------------------------------------- divergence
@pytest.mark.parametrize("n,k", [(2, 2), (4, 1), (2, 3)])
def test_direct_solution_is_discretely_divergence_free(n, k):
    S = Stokes(n, k)
    K = S.assemble()
    b = S.rhs(mf.sine_f, mf.sine_u)
    x = S.direct_solve(b, K)
    Bu = K[S.offsets[3]:, :S.offsets[3]] @ x[:S.offsets[3]]
    assert np.linalg.norm(Bu) <= 1e-12 * np.linalg.norm(b)


def test_mg_solution_is_discretely_divergence_free():
    """FGMRES + V-cycle to a residual of 1e-13: the pressure rows of the
    residual are -B u_h, so ||B u_h|| <= 1e-12 ||b||."""
    mg = Multigrid(4, 1)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    x, hist = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v), rtol=1e-13)
    Bu = K[S.offsets[3]:, :S.offsets[3]] @ x[:S.offsets[3]]
    assert np.linalg.norm(Bu) <= 1e-12 * np.linalg.norm(b)


# --------------------------------------------------------------------- Adam
def test_adam_matches_closed_sum_over_several_steps():
    """Kingma & Ba: m_t = (1 - b1) sum_i b1^(t-i) g_i, v_t likewise with g_i^2,
    bias-corrected by 1 - b^t.  Moments in exact rational arithmetic, over
    five steps with changing gradients."""
    b1, b2, lr, eps = Fraction(9, 10), Fraction(999, 1000), 1e-3, 1e-8
    gs = [Fraction(1), Fraction(-2), Fraction(1, 2), Fraction(3), Fraction(-1, 4)]
    p = [np.array([0.7])]
    m = [np.zeros(1)]
    v = [np.zeros(1)]
    expect = 0.7
    for t in range(1, len(gs) + 1):
        p, m, v = mlp.adam_step(p, [np.array([float(gs[t - 1])])], m, v, t=t, lr=lr, eps=eps)
        mt = (1 - b1) * sum(b1 ** (t - i) * gs[i - 1] for i in range(1, t + 1))
        vt = (1 - b2) * sum(b2 ** (t - i) * gs[i - 1] ** 2 for i in range(1, t + 1))
        assert abs(m[0][0] - float(mt)) <= 1e-15 * max(1.0, abs(float(mt)))
        assert abs(v[0][0] - float(vt)) <= 1e-15 * max(1.0, abs(float(vt)))
        mhat = float(mt / (1 - b1 ** t))
        vhat = float(vt / (1 - b2 ** t))
        expect -= lr * mhat / (np.sqrt(vhat) + eps)
        assert abs(p[0][0] - expect) <= 1e-13, t


def test_adam_constant_gradient_steps_are_lr_sign():
    """With bias correction, a constant gradient gives m_hat = g and
    v_hat = g^2 at every step, so each step moves by exactly lr sign(g)
    (eps = 0)."""
    rng = np.random.default_rng(4)
    g = [rng.normal(size=(4, 3))]
    p = [rng.normal(size=(4, 3))]
    m = [np.zeros((4, 3))]
    v = [np.zeros((4, 3))]
    lr = 2e-3
    for t in range(1, 8):
        newp, m, v = mlp.adam_step(p, g, m, v, t=t, lr=lr, eps=0.0)
        assert np.allclose(p[0] - newp[0], lr * np.sign(g[0]), rtol=1e-10, atol=0), t
        p = newp


# ------------------------------------------------- learned-solver callbacks
def _exact_normalized_map(mg, l, v):
    """D_out K_j^+ D_in of an interior patch: (F/h, G/h^2) -> (U, hP)."""
    lev = mg.levels[l]
    S, Pt, K = lev["S"], lev["patches"], lev["K"]
    nv = 3 * Pt.nvel
    d_in = np.concatenate([np.full(nv, S.h), np.full(Pt.npres, S.h ** 2)])
    d_out = np.concatenate([np.ones(nv), np.full(Pt.npres, S.h)])
    return d_out[:, None] * Pt.pinv(K, v) * d_in[None, :]


def test_learned_sweep_with_exact_map_equals_exact_sweep(monkeypatch):
    """The network replaced by the exact normalized map (the same matrix for
    every interior patch): the learned callback's scaling, unscaling,
    pressure projection and interior/boundary split reproduce Alg. 2."""
    n, k = 8, 1
    mg = Multigrid(n, k)
    l = len(mg.levels) - 1
    Mt = _exact_normalized_map(mg, l, np.array([3, 3, 3])).T
    monkeypatch.setattr(mlp, "forward", lambda params, X: (X @ Mt, None))
    S = mg.fine["S"]
    rng = np.random.default_rng(11)
    x0 = rng.uniform(-1, 1, S.ndof)
    b = rng.uniform(-1, 1, S.ndof)
    ref = mg.smooth(l, x0, b)
    got = mg.smooth(l, x0, b, local=mlp.learned_local(mg, None))
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_captured_pairs_follow_the_exact_map():
    n, k = 8, 1
    mg = Multigrid(n, k)
    l = len(mg.levels) - 1
    M = _exact_normalized_map(mg, l, np.array([2, 2, 2]))
    S = mg.fine["S"]
    b = np.random.default_rng(12).uniform(-1, 1, S.ndof)
    sink = []
    mg.smooth(l, np.zeros(S.ndof), b, local=mlp.capture_local(mg, sink, l))
    assert len(sink) == (n - 3) ** 3                   # interior patches: 2 <= v_d <= n-2
    for x, t in sink:
        assert abs(np.linalg.norm(x) - 1.0) <= 1e-14
        assert np.linalg.norm(M @ x - t) <= 1e-12 * np.linalg.norm(t)


# ---------------------------------------------------- contraction monitor
def _hist(rhos):
    h = [1.0]
    for r in rhos:
        h.append(h[-1] * r)
    return h


def test_monitor_synthetic_sequences():
    rho_ref = 0.02                                    # bound 0.04
    assert mlp.fallback_step(_hist([0.03, 0.02, 0.039]), rho_ref) == -1
    assert mlp.fallback_step(_hist([0.03, 0.02, 0.041, 0.01]), rho_ref) == 3
    assert mlp.fallback_step(_hist([0.05]), rho_ref) == 1
    assert mlp.fallback_step(_hist([0.25, 0.5]), 0.25) == 2           # the bound itself triggers
    assert mlp.fallback_step(_hist([1e-4, 2e-3]), 1e-4) == 2           # bound max(2e-4, 1e-3) = 1e-3 ...
    assert mlp.fallback_step(_hist([1e-4, 9e-4]), 1e-4) == -1          # ... and below it, no trigger
    assert mlp.fallback_step(_hist([0.5, 0.9, 1.2]), 0.0) == 3         # no reference: growth triggers
    assert mlp.fallback_step([1.0, 0.03, float("nan")], 0.02) == 2


def test_zeroed_network_triggers_within_two_steps():
    """A network whose output is identically zero leaves every interior patch
    uncorrected.  On 8^3 cells, k = 2, the first FGMRES step still contracts
    by about 0.011 (the coarse-grid correction and the exact solves on the
    boundary patches carry it; the plain method's first step gives 0.0094),
    but the second contracts by about 0.25, far above the bound
    2 rho_ref = 0.036: the monitor hands over at step 2."""
    n, k = 8, 2
    mg = Multigrid(n, k)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    _, h_plain = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v), rtol=1e-8)
    rho_ref = h_plain[-1] ** (1.0 / (len(h_plain) - 1))
    d = 3 * mg.fine["patches"].nvel + mg.fine["patches"].npres
    zero = [np.zeros((d, 8)), np.zeros(8), np.zeros((8, 8)), np.zeros(8), np.zeros((8, d)), np.zeros(d)]
    loc = mlp.learned_local(mg, zero)
    _, h = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v, local=loc), rtol=1e-8, maxit=3)
    assert mlp.fallback_step(h, rho_ref) == 2, (h, rho_ref)
    assert mlp.fallback_step(h_plain, rho_ref) == -1
