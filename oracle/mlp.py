"""Per-patch MLP local solver: forward, loss, backward and Adam in float64
(oracle; test infrastructure).

Not in the paper: a learned stand-in for the local solve of Sec. 3.2, trained
on (patch residual, exact local correction) pairs produced by the plain
smoother.  Network: x -> GELU(x W1 + b1) -> GELU(. W2 + b2) -> . W3 + b3 with
GELU(z) = z Phi(z) (Phi the standard normal CDF, written with erf), loss =
mean squared error over all entries, optimizer Adam (Kingma & Ba 2015).

Scaling of a patch problem (exact for interior patches): with A_j = h A^,
B_j = h^2 B^, the correction satisfies (U, h P) = K^+ (F / h, G / h^2) with a
level-independent K^.  The network therefore sees x = (F/h, G/h^2) / s and is
trained on t = (U, h P) / s, s = ||(F/h, G/h^2)||, which keeps the learned map
positively homogeneous like the exact one.
"""
import math

import numpy as np
from scipy.special import erf


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, X):
    """Returns the output and the cache (pre-activations, activations)."""
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    Y = H2 @ W3 + b3
    return Y, (X, Z1, H1, Z2, H2)


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(params, cache, Y, T):
    """Gradients of mse(Y, T) with respect to (W1, b1, W2, b2, W3, b3)."""
    W1, b1, W2, b2, W3, b3 = params
    X, Z1, H1, Z2, H2 = cache
    dY = 2.0 * (Y - T) / Y.size
    dW3 = H2.T @ dY
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * gelu_grad(Z2)
    dW2 = H1.T @ dZ2
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new params, m, v."""
    new_p, new_m, new_v = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1.0 - beta1) * g
        vi = beta2 * vi + (1.0 - beta2) * g * g
        mhat = mi / (1.0 - beta1 ** t)
        vhat = vi / (1.0 - beta2 ** t)
        new_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        new_m.append(mi)
        new_v.append(vi)
    return new_p, new_m, new_v


def normalize_pair(F, G, U, P, h):
    """Network input and target of one patch problem (see module doc)."""
    x = np.concatenate([F / h, G / h ** 2])
    s = np.linalg.norm(x)
    if s == 0:
        return np.zeros_like(x), np.zeros(len(U) + len(P)), 0.0
    return x / s, np.concatenate([U, h * P]) / s, s


def denormalize(y, s, nvel, h):
    """Correction (U, P) from a network output for input scale s."""
    return s * y[:nvel], s * y[nvel:] / h


def is_interior(Pt, v):
    """A patch whose 8 cells touch no boundary face (2 <= v_d <= n-2)."""
    return all(t == (0, 0) for t in Pt.patch_type(v))


def learned_local(mg, params):
    """Local-solver callback for Multigrid.smooth: the network on interior
    patches (scaled as in the module doc, patch pressure projected to zero
    coefficient mean), the pseudo-inverse elsewhere."""
    def local(l, v, rj):
        lev = mg.levels[l]
        S, Pt = lev["S"], lev["patches"]
        if not is_interior(Pt, v):
            return Pt.local_solve(lev["K"], v, rj)
        nv = 3 * Pt.nvel
        x, _, s = normalize_pair(rj[:nv], rj[nv:], np.zeros(nv), np.zeros(Pt.npres), S.h)
        if s == 0:
            return np.zeros_like(rj)
        y, _ = forward(params, x[None, :])
        U, P = denormalize(y[0], s, nv, S.h)
        # the exact correction is orthogonal to the kernel of K_j (constant patch
        # pressure); the learned one is projected the same way
        return np.concatenate([U, P - P.mean()])
    return local


def capture_local(mg, sink, level):
    """Local-solver callback that solves exactly (pseudo-inverse) and appends
    the normalized (input, target) pair of every interior patch of `level`
    to sink (a list), in the order the smoother visits them."""
    def local(l, v, rj):
        lev = mg.levels[l]
        S, Pt = lev["S"], lev["patches"]
        upd = Pt.local_solve(lev["K"], v, rj)
        if l == level and is_interior(Pt, v):
            nv = 3 * Pt.nvel
            x, t, _ = normalize_pair(rj[:nv], rj[nv:], upd[:nv], upd[nv:], S.h)
            sink.append((x, t))
        return upd
    return local


def fallback_step(history, rho_ref):
    """Contraction monitor of the learned local solver (not in the paper; the
    exact solver is the fallback).  history[0] = 1 and history[n] is the
    relative residual after outer step n.  The monitor looks at the
    contraction rho_n = history[n] / history[n-1] of every step and returns
    the first n at which it hands the rest of the solve to the exact local
    solver, or -1 if it never does.  The bound is max(2 rho_ref, 1e-3) when a
    reference contraction rho_ref > 0 of the plain method is known, else 1
    (no progress); a contraction that is not finite also triggers."""
    bound = max(2.0 * rho_ref, 1e-3) if rho_ref > 0 else 1.0
    for n in range(1, len(history)):
        rho = history[n] / history[n - 1] if history[n - 1] != 0 else float("nan")
        if not (rho < bound):
            return n
    return -1
