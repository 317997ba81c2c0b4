"""Seeded synthetic inputs (no discretization arithmetic): the only code the
tests, the benchmark and the oracle-side checks share.  NumPy PCG64."""
import numpy as np


def uniform_vector(n, seed, dtype=np.float64):
    """x ~ U[-1, 1]^n from PCG64(seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, int(n)).astype(dtype)


def fourier_modes(seed, n_modes=8, kmax=8):
    """Parameters of a random smooth field per velocity component:
    f_c(x) = sum_m a[c,m] cos(pi kappa[c,m] . x + theta[c,m]) with integer
    wavenumbers kappa in {1..kmax}^3, a ~ U[-1, 1], theta ~ U[0, 2 pi)."""
    g = np.random.default_rng(seed)
    kappa = g.integers(1, kmax + 1, size=(3, n_modes, 3))
    amp = g.uniform(-1.0, 1.0, size=(3, n_modes))
    theta = g.uniform(0.0, 2 * np.pi, size=(3, n_modes))
    return kappa, amp, theta
