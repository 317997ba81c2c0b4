"""1D reference data on the unit interval [0, 1] (oracle; test infrastructure).

The Raviart-Thomas element RT_k of Sec. 2.1 is a tensor product of 1D
polynomial spaces: degree k+1 in the component's own ("parallel") direction,
where the normal component is continuous across faces, and degree k in the
other ("orthogonal") directions, where it is discontinuous (Fig. RT2 and the
text around it).  The pressure is discontinuous Q_k.

The paper does not name the nodal bases.  Reading used here: the continuous
direction uses Lagrange polynomials on the k+2 Gauss-Lobatto points (so that
the end nodes carry the normal trace and are shared between neighbouring
cells); the discontinuous directions and the pressure use Lagrange
polynomials on the k+1 Gauss points.
"""
import numpy as np


def gauss(npts):
    """Gauss-Legendre rule with ``npts`` points on [0, 1]: (points, weights)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto_points(npts):
    """Gauss-Lobatto points (``npts`` >= 2, endpoints included) on [0, 1].

    The interior points are the roots of P'_{npts-1}, the derivative of the
    Legendre polynomial of degree npts-1.
    """
    if npts < 2:
        raise ValueError("Gauss-Lobatto needs at least two points")
    if npts == 2:
        inner = np.array([])
    else:
        c = np.zeros(npts)
        c[-1] = 1.0
        inner = np.sort(np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c)).real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def lagrange_values(nodes, x):
    """V[i, q] = l_i(x_q) for the Lagrange basis on ``nodes`` (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(nodes)
    V = np.ones((m, len(x)))
    for i in range(m):
        for j in range(m):
            if j != i:
                V[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[i, q] = l_i'(x_q), by the product rule applied to the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(nodes)
    D = np.zeros((m, len(x)))
    for i in range(m):
        for r in range(m):
            if r == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[r]))
            for j in range(m):
                if j != i and j != r:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return D


class Basis1D:
    """The two 1D bases of RT_k / Q_k for degree ``k``.

    ``dg``:   Lagrange on the k+1 Gauss points (discontinuous directions, pressure)
    ``cont``: Lagrange on the k+2 Gauss-Lobatto points (continuous direction)
    """

    def __init__(self, k):
        if k < 0:
            raise ValueError("degree must be >= 0")
        self.k = k
        self.dg_nodes, self.dg_weights = gauss(k + 1)
        if k == 0:
            self.cont_nodes = np.array([0.0, 1.0])
        else:
            self.cont_nodes = gauss_lobatto_points(k + 2)

    def values(self, kind, x):
        nodes = self.dg_nodes if kind == "dg" else self.cont_nodes
        return lagrange_values(nodes, x)

    def derivatives(self, kind, x):
        nodes = self.dg_nodes if kind == "dg" else self.cont_nodes
        return lagrange_derivatives(nodes, x)

    def size(self, kind):
        return self.k + 1 if kind == "dg" else self.k + 2
