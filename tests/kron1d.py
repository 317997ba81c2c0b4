"""An independent route to the global operator, used only to pin the oracle:
1D matrices assembled from 1D integrals and 1D face terms, combined by
Kronecker products (the separable form of Sec. 2.2 and of Eqs. block_A/b for
the patch matrices, extended to 3D and to the whole mesh).

The oracle assembles K by 3D quadrature of the bilinear form; this module
never looks at that code.  Agreement of the two pins both.

1D forms on [0,1] with n cells, h = 1/n, gamma = 2 (k+1)^2 / h:

* DG direction: M_d(u, v) = int u v;  L_d(u, v) = sum_cells int u' v'
  + sum_interior_faces (gamma [u][v] - {{u'}}[v] - [u]{{v'}})
  + sum_boundary (2 gamma u v - d_n u v - u d_n v), the 1D restriction of
  Eq. bilinear.
* continuous direction: M_c, L_c = int u v, int u' v' on the continuous
  piecewise polynomials with shared nodes, restricted to interior nodes
  (the normal component has no jumps, hence no face terms).
* D(q, u) = int q u' (pressure test, continuous trial).

3D (x fastest, so a matrix acting on (z, y, x) is kron(Z, kron(Y, X))):
  A_x = Mz_d Y_d L_c^x + M_d L_d M_c + L_d M_d M_c, and cyclically,
  B_x = -kron(M_d, kron(M_d, D)), etc.
"""
import numpy as np
import scipy.sparse as sp

from oracle.fe1d import gauss, gauss_lobatto_points, lagrange_values, lagrange_derivatives


def ref_1d(k):
    xg, _ = gauss(k + 1)
    xl = gauss_lobatto_points(k + 2)
    xq, wq = gauss(k + 2)
    Vd, Dd = lagrange_values(xg, xq), lagrange_derivatives(xg, xq)
    Vc, Dc = lagrange_values(xl, xq), lagrange_derivatives(xl, xq)
    W = np.diag(wq)
    out = dict(
        Md=Vd @ W @ Vd.T, Kd=Dd @ W @ Dd.T,
        Mc=Vc @ W @ Vc.T, Kc=Dc @ W @ Dc.T,
        D=Vd @ W @ Dc.T,                      # (k+1) x (k+2): int l_a phi_b'
        eL=lagrange_values(xg, [0.0])[:, 0], eR=lagrange_values(xg, [1.0])[:, 0],
        dL=lagrange_derivatives(xg, [0.0])[:, 0], dR=lagrange_derivatives(xg, [1.0])[:, 0],
    )
    return out


def global_1d(n, k, penalty_factor=2.0):
    h = 1.0 / n
    gam = penalty_factor * (k + 1) ** 2 / h
    r = ref_1d(k)
    m = k + 1
    N1 = n * m
    Md = np.zeros((N1, N1))
    Ld = np.zeros((N1, N1))
    for i in range(n):
        s = slice(i * m, (i + 1) * m)
        Md[s, s] += h * r["Md"]
        Ld[s, s] += r["Kd"] / h
    for f in range(1, n):                    # face between cells f-1 (minus) and f (plus)
        J = np.zeros(N1)
        Av = np.zeros(N1)
        J[(f - 1) * m:f * m] += r["eR"]
        J[f * m:(f + 1) * m] -= r["eL"]
        Av[(f - 1) * m:f * m] += 0.5 * r["dR"] / h
        Av[f * m:(f + 1) * m] += 0.5 * r["dL"] / h
        Ld += gam * np.outer(J, J) - np.outer(J, Av) - np.outer(Av, J)
    for side in (0, 1):
        V = np.zeros(N1)
        Dn = np.zeros(N1)
        if side == 0:
            V[:m] = r["eL"]
            Dn[:m] = -r["dL"] / h
        else:
            V[-m:] = r["eR"]
            Dn[-m:] = r["dR"] / h
        Ld += 2 * gam * np.outer(V, V) - np.outer(V, Dn) - np.outer(Dn, V)
    Mc = np.zeros((N1 + 1, N1 + 1))
    Lc = np.zeros((N1 + 1, N1 + 1))
    D = np.zeros((N1, N1 + 1))
    for i in range(n):
        s = slice(i * m, i * m + k + 2)
        Mc[s, s] += h * r["Mc"]
        Lc[s, s] += r["Kc"] / h
        D[i * m:(i + 1) * m, s] += r["D"]
    inner = slice(1, N1)
    return dict(Md=Md, Ld=Ld, Mc=Mc[inner, inner], Lc=Lc[inner, inner], D=D[:, inner], h=h, gamma=gam)


def kron3(Z, Y, X):
    return sp.kron(sp.csr_matrix(Z), sp.kron(sp.csr_matrix(Y), sp.csr_matrix(X)))


def global_operator(n, k):
    g = global_1d(n, k)
    Md, Ld, Mc, Lc, D = g["Md"], g["Ld"], g["Mc"], g["Lc"], g["D"]
    Ax = kron3(Md, Md, Lc) + kron3(Md, Ld, Mc) + kron3(Ld, Md, Mc)
    Ay = kron3(Md, Lc, Md) + kron3(Md, Mc, Ld) + kron3(Ld, Mc, Md)
    Az = kron3(Lc, Md, Md) + kron3(Mc, Ld, Md) + kron3(Mc, Md, Ld)
    Bx = -kron3(Md, Md, D)
    By = -kron3(Md, D, Md)
    Bz = -kron3(D, Md, Md)
    A = sp.block_diag([Ax, Ay, Az])
    B = sp.hstack([Bx, By, Bz])
    return sp.bmat([[A, B.T], [B, None]]).tocsr()


def patch_1d(n, k, v):
    """Restrictions of the global 1D matrices to the windows of the patch at
    vertex index v (one direction): 2k+2 DG indices and 2k+1 interior nodes
    starting at (v-1)(k+1)."""
    g = global_1d(n, k)
    base = (v - 1) * (k + 1)
    wd = slice(base, base + 2 * k + 2)
    wc = slice(base, base + 2 * k + 1)
    return dict(Md=g["Md"][wd, wd], Ld=g["Ld"][wd, wd], Mc=g["Mc"][wc, wc], Lc=g["Lc"][wc, wc],
                D=g["D"][wd, wc])
