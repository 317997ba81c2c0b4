"""Pins of the oracle's MLP pieces (CPU): GELU against closed values and the
normal CDF, gradients against central finite differences, Adam's first step
(|step| = lr for every entry with a nonzero gradient), MSE of a constant
shift, and the scaling of the patch problem (the normalized exact map is the
same on two levels)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp
from oracle.stokes import Stokes
from oracle.patches import Patches


def test_gelu_values():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0, 6.0])
    assert abs(mlp.gelu(np.array([0.0]))[0]) == 0.0
    assert np.allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-14, atol=1e-15)
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    e = 1e-6
    assert np.allclose(mlp.gelu_grad(z), (mlp.gelu(z + e) - mlp.gelu(z - e)) / (2 * e), atol=1e-8)


def _params(rng, sizes):
    p = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        p += [rng.normal(0, 1 / math.sqrt(a), (a, b)), rng.normal(0, 0.1, b)]
    return p


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 5, 6, 4]
    params = _params(rng, sizes)
    X = rng.normal(size=(9, 7))
    T = rng.normal(size=(9, 4))
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T)
    e = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + e
            lp = mlp.mse(mlp.forward(params, X)[0], T)
            flat[idx] = old - e
            lm = mlp.mse(mlp.forward(params, X)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * e)
            assert abs(fd - g.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (pi, idx)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(1)
    p = [rng.normal(size=(3, 4))]
    g = [rng.normal(size=(3, 4))]
    m = [np.zeros((3, 4))]
    v = [np.zeros((3, 4))]
    lr = 1e-3
    newp, _, _ = mlp.adam_step(p, g, m, v, t=1, lr=lr, eps=0.0)
    assert np.allclose(p[0] - newp[0], lr * np.sign(g[0]), rtol=1e-12)


def test_mse_constant_shift():
    Y = np.zeros((5, 3))
    assert mlp.mse(Y + 2.0, Y) == 4.0


def test_normalized_exact_map_is_level_independent():
    """Interior patches of two levels: the exact map (F/h, G/h^2) -> (U, hP)
    is the same matrix, so one network serves every level."""
    k = 1
    maps = []
    for n in (4, 8):
        S = Stokes(n, k)
        K = S.assemble()
        Pt = Patches(S)
        v = np.array([2, 2, 2])
        Kp = Pt.pinv(K, v)
        nv = 3 * Pt.nvel
        D_in = np.diag(np.concatenate([np.full(nv, S.h), np.full(Pt.npres, S.h ** 2)]))   # (F, G) from (F/h, G/h^2)
        D_out = np.diag(np.concatenate([np.ones(nv), np.full(Pt.npres, S.h)]))           # (U, hP) from (U, P)
        maps.append(D_out @ Kp @ D_in)
    assert np.abs(maps[0] - maps[1]).max() <= 1e-10 * np.abs(maps[0]).max()


def test_normalize_roundtrip():
    rng = np.random.default_rng(2)
    F, G, U, P = rng.normal(size=5), rng.normal(size=3), rng.normal(size=5), rng.normal(size=3)
    h = 0.25
    x, t, s = mlp.normalize_pair(F, G, U, P, h)
    assert abs(np.linalg.norm(x) - 1.0) < 1e-14
    U2, P2 = mlp.denormalize(t, s, 5, h)
    assert np.allclose(U2, U) and np.allclose(P2, P)
