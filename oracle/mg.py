"""Multigrid for the discrete Stokes problem (oracle; test infrastructure,
float64): transfers, the colourized vertex-patch smoother, the V-cycle and
right-preconditioned restarted FGMRES.

* Hierarchy (Sec. 3): uniform refinement, levels with n = 2^l cells per
  direction; every level is discretized anew with its own h and gamma.
* Prolongation (Sec. 3): the canonical embedding X_{l-1} -> X_l.  With nodal
  bases its matrix holds the coarse basis functions evaluated at the fine
  DoF support points.  Restriction: its transpose (the restriction of
  residual functionals).
* Coarsest level: the pseudo-inverse of K_0 (P_0^{-1} = A_0^{-1} of Sec. 3,
  K_0 being singular only through the constant pressure).
* Smoother (Alg. 2): colours in sequence; for each colour the global
  residual r = b - K x is formed once and every patch of that colour adds
  R_j^T K_j^+ R_j r.
* V-cycle (Sec. 3): pre-smooth, coarse-grid correction, post-smooth.
* Outer solver: GMRES preconditioned by the V-cycle (Sec. 3.3), written as
  flexible GMRES (Saad 1993) with restart, modified Gram-Schmidt and Givens
  rotations, stopping on the Euclidean norm of the residual relative to the
  right-hand side.
"""
import numpy as np
import scipy.sparse as sp

from .stokes import Stokes
from .patches import Patches


def prolongation(Sc, Sf):
    """Sparse matrix of the canonical embedding from Sc (n cells) into Sf
    (2n cells)."""
    assert Sf.n == 2 * Sc.n and Sf.k == Sc.k
    k = Sf.k
    H = Sc.h
    rows, cols, vals = [], [], []
    xg = Sf.basis.dg_nodes
    xl = Sf.basis.cont_nodes
    dg_coord = (np.repeat(np.arange(Sf.n), k + 1) + np.tile(xg, Sf.n)) * Sf.h
    cont_coord = np.concatenate([(i + xl[:-1]) * Sf.h for i in range(Sf.n)] + [[1.0]])[1:-1]

    def lift(coords, c):
        # fine support points of one component (x fastest) -> coarse cell and reference coordinate
        Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
        P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        cell = np.clip(np.floor(P / H).astype(np.int64), 0, Sc.n - 1)
        ref = P / H - cell
        return cell, ref

    for c in range(4):
        coords = [dg_coord] * 3
        if c < 3:
            coords[c] = cont_coord
        cell, ref = lift(coords, c)
        nfine = cell.shape[0]
        fine_idx = Sf.offsets[c] + np.arange(nfine)
        # evaluate the coarse local basis of this component at each point
        kinds = ["dg"] * 3
        if c < 3:
            kinds[c] = "cont"
        sizes = [Sc.basis.size(kd) for kd in kinds]
        V1 = [Sc.basis.values(kinds[d], ref[:, d]) for d in range(3)]     # (size_d, nfine)
        tup = Sc.local_tuples(sizes)
        vals_c = np.array([V1[0][b0] * V1[1][b1] * V1[2][b2] for (b0, b1, b2) in tup]).T  # (nfine, nloc)
        gidx = Sc.vel_global(c, cell) if c < 3 else Sc.pres_global(cell)
        ok = (gidx >= 0) & (np.abs(vals_c) > 0)
        rows.append(np.broadcast_to(fine_idx[:, None], gidx.shape)[ok])
        cols.append(gidx[ok])
        vals.append(vals_c[ok])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Sf.ndof, Sc.ndof)).tocsr()
    P.sum_duplicates()
    return P


class Multigrid:
    """Level hierarchy n = 1, 2, 4, ..., n_fine (or from ``n_coarse``)."""

    def __init__(self, n_fine, k, n_coarse=1, penalty_factor=2.0, local_solver="pinv"):
        self.levels = []
        n = n_coarse
        while n <= n_fine:
            S = Stokes(n, k, penalty_factor)
            K = S.assemble()
            Pt = Patches(S, local_solver) if n >= 2 else None
            self.levels.append(dict(S=S, K=K, patches=Pt))
            n *= 2
        assert self.levels[-1]["S"].n == n_fine, "n_fine must be n_coarse * 2^L"
        self.P = [None] + [prolongation(self.levels[l - 1]["S"], self.levels[l]["S"])
                           for l in range(1, len(self.levels))]
        self._K0_pinv = None

    @property
    def K0_pinv(self):
        """Dense pseudo-inverse of the coarsest matrix (computed on first use)."""
        if self._K0_pinv is None:
            K0 = self.levels[0]["K"].toarray()
            lam, Q = np.linalg.eigh(K0)
            drop = np.argmin(np.abs(lam))
            keep = np.ones(len(lam), dtype=bool)
            keep[drop] = False
            self._K0_pinv = (Q[:, keep] / lam[keep]) @ Q[:, keep].T
        return self._K0_pinv

    @property
    def fine(self):
        return self.levels[-1]

    def smooth(self, l, x, b, local=None):
        """One sweep of Alg. 2 on level l (colours 0..7 ascending).  ``local``
        optionally replaces the pinv local solve: local(l, v, r_j) -> update."""
        lev = self.levels[l]
        K, Pt = lev["K"], lev["patches"]
        x = np.array(x, dtype=np.float64)
        for c in range(8):
            verts = Pt.verts[Pt.colour == c]
            if len(verts) == 0:
                continue
            r = b - K @ x
            dx = np.zeros_like(x)
            for v in verts:
                idx = Pt.dofs(v)
                rj = r[idx]
                upd = Pt.local_solve(K, v, rj) if local is None else local(l, v, rj)
                dx[idx] += upd
            x += dx
        return x

    def vcycle(self, b, l=None, pre=1, post=1, local=None):
        """x = P_l^{-1} b starting from x = 0 (Sec. 3)."""
        if l is None:
            l = len(self.levels) - 1
        if l == 0:
            return self.K0_pinv @ b
        x = np.zeros_like(b)
        for _ in range(pre):
            x = self.smooth(l, x, b, local)
        r = b - self.levels[l]["K"] @ x
        ec = self.vcycle(self.P[l].T @ r, l - 1, pre, post, local)
        x = x + self.P[l] @ ec
        for _ in range(post):
            x = self.smooth(l, x, b, local)
        return x


def fgmres(apply_K, b, precond, rtol=1e-8, restart=30, maxit=200):
    """Right-preconditioned restarted flexible GMRES, x0 = 0.
    Returns (x, history of ||b - K x_j|| / ||b||)."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    if nb == 0:
        return x, hist
    it = 0
    while it < maxit:
        r = b - apply_K(x)
        beta = np.linalg.norm(r)
        if beta / nb <= rtol:
            break
        V = [r / beta]
        Z = []
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_done = 0
        for j in range(restart):
            z = precond(V[j])
            Z.append(z)
            w = apply_K(z)
            for i in range(j + 1):
                Hm[i, j] = w @ V[i]
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            V.append(w / Hm[j + 1, j] if Hm[j + 1, j] != 0 else w)
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j] = Hm[j, j] / den
            sn[j] = Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= rtol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(Hm[:j_done, :j_done]), g[:j_done])
        for i in range(j_done):
            x = x + y[i] * Z[i]
        if hist[-1] <= rtol:
            break
    return x, hist


def fractional_iterations(hist):
    """Fractional iteration count of Sec. 3.3: the number of steps that the
    average contraction rbar = (||r_n|| / ||r_0||)^(1/n) needs to reduce the
    residual by 1e-8, nu = -8 / log10(rbar).  (The printed formula reads as a
    product, which cannot be meant: it would make faster convergence give a
    larger count; the quotient is the reading used.)"""
    n = len(hist) - 1
    rbar = (hist[-1] / hist[0]) ** (1.0 / n)
    return -8.0 / np.log10(rbar)
