"""Analytic test problems for the Stokes equations of Eq. model (test data,
no discretization arithmetic).

* ``poly``: u = (x(1-x)(2y-1), -(2x-1)y(1-y), 0), p = (x-1/2)(y-1/2)(z-1/2).
  u lies in RT_k for every k >= 1, is divergence free and has u.n = 0 on the
  boundary (nonzero tangential trace); p lies in Q_k with zero mean.  The
  discrete solution must reproduce it exactly.
* ``sine``: u = curl(psi (1,1,1)), psi = sin(pi x) sin(pi y) sin(pi z),
  p = cos(pi x) cos(pi y) cos(pi z) (zero mean).  u.n = 0 on the boundary,
  -Laplace(u) = 3 pi^2 u, f = 3 pi^2 u + grad p.  The tangential trace of u is
  not zero; it enters through the boundary (Nitsche) terms of the bilinear
  form.
* ``pressure_only``: u = 0, p = (x-1/2)^2 (y-1/2) - mean, f = grad p: the
  discrete solution is (0, p) exactly for k >= 2.
"""
import numpy as np

PI = np.pi


def poly_u(x, y, z):
    return np.array([x * (1 - x) * (2 * y - 1), -(2 * x - 1) * y * (1 - y), 0.0 * x])


def poly_p(x, y, z):
    return (x - 0.5) * (y - 0.5) * (z - 0.5)


def poly_f(x, y, z):
    # -Laplace(u) + grad(p)
    return np.array([2 * (2 * y - 1) + (y - 0.5) * (z - 0.5),
                     -2 * (2 * x - 1) + (x - 0.5) * (z - 0.5),
                     (x - 0.5) * (y - 0.5) + 0.0 * z])


def sine_u(x, y, z):
    sx, sy, sz = np.sin(PI * x), np.sin(PI * y), np.sin(PI * z)
    cx, cy, cz = np.cos(PI * x), np.cos(PI * y), np.cos(PI * z)
    return PI * np.array([sx * (cy * sz - sy * cz), sy * (sx * cz - cx * sz), sz * (cx * sy - sx * cy)])


def sine_p(x, y, z):
    return np.cos(PI * x) * np.cos(PI * y) * np.cos(PI * z)


def sine_f(x, y, z):
    sx, sy, sz = np.sin(PI * x), np.sin(PI * y), np.sin(PI * z)
    cx, cy, cz = np.cos(PI * x), np.cos(PI * y), np.cos(PI * z)
    return 3 * PI ** 2 * sine_u(x, y, z) - PI * np.array([sx * cy * cz, cx * sy * cz, cx * cy * sz])


def ponly_u(x, y, z):
    return np.array([0.0 * x, 0.0 * x, 0.0 * x])


def ponly_p(x, y, z):
    return (x - 0.5) ** 2 * (y - 0.5) - 0.0 * z


def ponly_f(x, y, z):
    return np.array([2 * (x - 0.5) * (y - 0.5), (x - 0.5) ** 2 + 0.0 * y, 0.0 * z])


def fourier_force(seed, n_modes=8):
    """The random smooth force of synth.fourier_modes(seed), evaluated
    pointwise: f_c = sum_m a cos(pi kappa . x + theta)."""
    from paper_2410_09497_amd.synth import fourier_modes
    kappa, amp, theta = fourier_modes(seed, n_modes=n_modes)

    def f(x, y, z):
        out = []
        for c in range(3):
            v = np.zeros_like(np.asarray(x, dtype=float))
            for m in range(n_modes):
                kx, ky, kz = kappa[c, m]
                v = v + amp[c, m] * np.cos(np.pi * (kx * x + ky * y + kz * z) + theta[c, m])
            out.append(v)
        return np.array(out)
    return f
