"""Pins of the oracle's 1D data against closed forms (CPU)."""
import numpy as np
import pytest

from oracle.fe1d import gauss, gauss_lobatto_points, lagrange_values, lagrange_derivatives, Basis1D


def test_gauss_two_points_closed_form():
    x, w = gauss(2)
    s = 1.0 / np.sqrt(3.0)
    assert np.allclose(x, [(1 - s) / 2, (1 + s) / 2], atol=1e-15)
    assert np.allclose(w, [0.5, 0.5], atol=1e-15)


def test_gauss_lobatto_closed_forms():
    assert np.allclose(gauss_lobatto_points(3), [0.0, 0.5, 1.0], atol=1e-15)
    # 4 points: +-1/sqrt(5) on [-1, 1]
    s = 1.0 / np.sqrt(5.0)
    assert np.allclose(gauss_lobatto_points(4), [0.0, (1 - s) / 2, (1 + s) / 2, 1.0], atol=1e-15)


@pytest.mark.parametrize("npts", range(1, 8))
def test_gauss_exactness(npts):
    x, w = gauss(npts)
    for m in range(2 * npts):
        assert abs(w @ x ** m - 1.0 / (m + 1)) < 1e-14
    # and not exact one degree above (the rule is not over-exact)
    m = 2 * npts
    assert abs(w @ x ** m - 1.0 / (m + 1)) > 1e-11


@pytest.mark.parametrize("k", range(1, 6))
def test_lagrange_delta_and_partition(k):
    b = Basis1D(k)
    for kind in ("dg", "cont"):
        nodes = b.dg_nodes if kind == "dg" else b.cont_nodes
        V = lagrange_values(nodes, nodes)
        assert np.allclose(V, np.eye(len(nodes)), atol=1e-14)
        xs = np.linspace(0, 1, 17)
        assert np.allclose(b.values(kind, xs).sum(axis=0), 1.0, atol=1e-13)
        assert np.allclose(b.derivatives(kind, xs).sum(axis=0), 0.0, atol=1e-11)


@pytest.mark.parametrize("k", range(1, 6))
def test_derivative_matches_finite_difference(k):
    b = Basis1D(k)
    xs = np.linspace(0.05, 0.95, 9)
    e = 1e-6
    for kind in ("dg", "cont"):
        fd = (b.values(kind, xs + e) - b.values(kind, xs - e)) / (2 * e)
        assert np.allclose(b.derivatives(kind, xs), fd, atol=1e-6)


@pytest.mark.parametrize("k", range(1, 6))
def test_dg_mass_is_diagonal(k):
    """Gauss-point Lagrange polynomials of degree k are orthogonal: the
    (k+2)-point Gauss rule integrates l_a l_b exactly, and the (k+1)-point
    rule, exact to degree 2k+1, evaluates it as w_a delta_ab."""
    b = Basis1D(k)
    xq, wq = gauss(k + 2)
    V = b.values("dg", xq)
    M = V @ np.diag(wq) @ V.T
    assert np.allclose(M, np.diag(b.dg_weights), atol=1e-15)
