"""The method in two dimensions (oracle; test infrastructure, float64): the
discrete Stokes problem of Sec. 2 on n^2 squares of the unit square, the
vertex-patch smoother of Sec. 3.1 with pseudo-inverse local solves (the
"Direct solver" of Sec. 3.3), the canonical-embedding transfers and the
V-cycle of Sec. 3, for the 2D workload of Table 1 (exact-2d).

Everything follows the 3D oracle (``stokes``, ``patches``, ``mg``) with one
direction less; the FGMRES and the fractional iteration count are the 3D
module's, which do not depend on the dimension.

* Space: RT_k velocity (the normal component continuous on Gauss-Lobatto
  points, k+2 per cell in its own direction; the tangential direction and the
  pressure discontinuous on k+1 Gauss points), u.n = 0 built in, DG Q_k
  pressure.  Layout [u_x | u_y | p]; component c is a lexicographic grid, x
  fastest, (N1-1) interior continuous nodes in direction c and N1 = n(k+1)
  discontinuous indices in the other; p is N1 x N1.
* Operator (Eq. bilinear, Eq. weak_form): cell term (grad u, grad v), interior
  edges gamma [u].[v] - {{d_n u}}.[v] - [u].{{d_n v}}, boundary edges
  2 gamma <u, v> - <d_n u, v> - <u, d_n v>, gamma = 2 (k+1)^2 / h, and
  B_{PX} = -(psi_P, div phi_X); Gauss quadrature with k+2 points per
  direction (exact for every term).
* Patches: one per interior vertex, the 4 cells around it; 4 colours by
  vertex parity; the patch space holds every DoF supported inside the patch
  (the normal nodes on the patch boundary excluded).
* Right-hand side of Sec. 3.3: u = (d_y psi, -d_x psi), psi = phi(x) phi(y),
  p = cos(2 pi x) cos(2 pi y), phi(x) = x^2 (x-1)^2 exp(-(x-mu)^2 / sigma^2)
  / sqrt(2 pi sigma^2).  The paper does not give mu and sigma; they are
  arguments here.  phi and phi' vanish at 0 and 1, so u = 0 on the boundary
  and the right-hand side is (f, phi) alone, f = -Laplace(u) + grad(p).
"""
from math import comb

import numpy as np
import scipy.sparse as sp

from .fe1d import Basis1D, gauss


def _square_points(x1d, w1d):
    """2D tensor points (x fastest) and weights on the unit square."""
    n = len(x1d)
    P = np.array([(x1d[a], x1d[b]) for b in range(n) for a in range(n)])
    W = np.array([w1d[a] * w1d[b] for b in range(n) for a in range(n)])
    return P, W


def _edge_points(d, t1d, w1d, coord):
    """Points on the reference edge x_d = coord, and their weights."""
    P = np.zeros((len(t1d), 2))
    P[:, d] = coord
    P[:, 1 - d] = t1d
    return P, np.asarray(w1d, dtype=np.float64)


class Stokes2D:
    """Discrete Stokes operator on n^2 cells with RT_k x DG Q_k."""

    def __init__(self, n, k, penalty_factor=2.0):
        if n < 1 or k < 1:
            raise ValueError("need n >= 1 and k >= 1")
        self.n, self.k = n, k
        self.h = 1.0 / n
        self.N1 = n * (k + 1)
        self.nc = (self.N1 - 1) * self.N1
        self.npres = self.N1 ** 2
        self.ndof = 2 * self.nc + self.npres
        self.offsets = (0, self.nc, 2 * self.nc)
        self.gamma = penalty_factor * (k + 1) ** 2 / self.h
        self.basis = Basis1D(k)
        self._local = None

    def vel_sizes(self, c):
        s = [self.k + 1] * 2
        s[c] = self.k + 2
        return s

    @staticmethod
    def local_tuples(sizes):
        return [(b0, b1) for b1 in range(sizes[1]) for b0 in range(sizes[0])]

    def vel_global(self, c, cells):
        """Global indices (ncells, nloc) of component c's local basis on the
        cells; -1 marks an eliminated boundary normal node."""
        k, N1 = self.k, self.N1
        cells = np.atleast_2d(cells)
        tup = np.array(self.local_tuples(self.vel_sizes(c)))
        idx, ext = [], []
        valid = np.ones((cells.shape[0], tup.shape[0]), dtype=bool)
        for d in range(2):
            pos = cells[:, d:d + 1] * (k + 1) + tup[None, :, d]
            if d == c:
                valid &= (pos > 0) & (pos < N1)
                idx.append(pos - 1)
                ext.append(N1 - 1)
            else:
                idx.append(pos)
                ext.append(N1)
        g = self.offsets[c] + idx[0] + ext[0] * idx[1]
        return np.where(valid, g, -1)

    def pres_global(self, cells):
        k, N1 = self.k, self.N1
        cells = np.atleast_2d(cells)
        tup = np.array(self.local_tuples([k + 1] * 2))
        pos = [cells[:, d:d + 1] * (k + 1) + tup[None, :, d] for d in range(2)]
        return self.offsets[2] + pos[0] + N1 * pos[1]

    def all_cells(self):
        i0, i1 = np.meshgrid(np.arange(self.n), np.arange(self.n), indexing="ij")
        return np.stack([i0.ravel(), i1.ravel()], axis=1)

    def eval_vel(self, c, P):
        kinds = ["dg", "dg"]
        kinds[c] = "cont"
        V1 = [self.basis.values(kinds[d], P[:, d]) for d in range(2)]
        D1 = [self.basis.derivatives(kinds[d], P[:, d]) for d in range(2)]
        tup = self.local_tuples(self.vel_sizes(c))
        val = np.array([V1[0][b0] * V1[1][b1] for (b0, b1) in tup])
        grad = np.array([[D1[0][b0] * V1[1][b1] for (b0, b1) in tup],
                         [V1[0][b0] * D1[1][b1] for (b0, b1) in tup]])
        return val, grad

    def eval_pres(self, P):
        V1 = [self.basis.values("dg", P[:, d]) for d in range(2)]
        return np.array([V1[0][b0] * V1[1][b1] for (b0, b1) in self.local_tuples([self.k + 1] * 2)])

    def local_matrices(self):
        if self._local is not None:
            return self._local
        k, h, gam = self.k, self.h, self.gamma
        xq, wq = gauss(k + 2)
        P, W = _square_points(xq, wq)
        W = W * h ** 2
        Q = self.eval_pres(P)
        cell_A, cell_B = [], []
        for c in range(2):
            _, G = self.eval_vel(c, P)
            G = G / h
            cell_A.append(sum(G[e] @ (W[:, None] * G[e].T) for e in range(2)))
            cell_B.append(-(Q @ (W[:, None] * G[c].T)))
        face, bface = {}, {}
        for d in range(2):
            Pm, Wf = _edge_points(d, xq, wq, 1.0)
            Pp, _ = _edge_points(d, xq, wq, 0.0)
            Wf = Wf * h
            for c in range(2):
                Vm, Gm = self.eval_vel(c, Pm)
                Vp, Gp = self.eval_vel(c, Pp)
                J = np.concatenate([Vm, -Vp])
                Av = 0.5 * np.concatenate([Gm[d] / h, Gp[d] / h])
                JW = J * Wf[None, :]
                face[(d, c)] = gam * JW @ J.T - JW @ Av.T - (Av * Wf[None, :]) @ J.T
                for side in (0, 1):
                    Pb, _ = _edge_points(d, xq, wq, float(side))
                    Vb, Gb = self.eval_vel(c, Pb)
                    Nb = (1.0 if side == 1 else -1.0) * Gb[d] / h
                    VW = Vb * Wf[None, :]
                    bface[(d, side, c)] = 2.0 * gam * VW @ Vb.T - VW @ Nb.T - (Nb * Wf[None, :]) @ Vb.T

        def clean(M):
            M = M.copy()
            M[np.abs(M) < 1e-12 * np.abs(M).max()] = 0.0
            return M

        self._local = dict(cell_A=[clean(M) for M in cell_A], cell_B=[clean(M) for M in cell_B],
                           face={key: clean(M) for key, M in face.items()},
                           bface={key: clean(M) for key, M in bface.items()})
        return self._local

    def blocks(self):
        L = self.local_matrices()
        n = self.n
        cells = self.all_cells()
        P = self.pres_global(cells)
        for c in range(2):
            R = self.vel_global(c, cells)
            yield R, R, L["cell_A"][c]
            yield P, R, L["cell_B"][c]
            yield R, P, L["cell_B"][c].T
        for d in range(2):
            e = np.zeros(2, dtype=int)
            e[d] = 1
            minus = cells[cells[:, d] < n - 1]
            plus = minus + e
            lo = cells[cells[:, d] == 0]
            hi = cells[cells[:, d] == n - 1]
            for c in range(2):
                R = np.concatenate([self.vel_global(c, minus), self.vel_global(c, plus)], axis=1)
                if R.shape[0]:
                    yield R, R, L["face"][(d, c)]
                Rl = self.vel_global(c, lo)
                yield Rl, Rl, L["bface"][(d, 0, c)]
                Rh = self.vel_global(c, hi)
                yield Rh, Rh, L["bface"][(d, 1, c)]

    def assemble(self):
        rows, cols, vals = [], [], []
        for R, C, M in self.blocks():
            nzr, nzc = np.nonzero(M)
            Rr, Cc = R[:, nzr], C[:, nzc]
            V = np.broadcast_to(M[nzr, nzc], Rr.shape)
            ok = (Rr >= 0) & (Cc >= 0)
            rows.append(Rr[ok])
            cols.append(Cc[ok])
            vals.append(V[ok])
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.ndof, self.ndof)).tocsr()
        K.sum_duplicates()
        return K

    def rhs(self, f, extra=2):
        """(f, phi) for every velocity basis function by Gauss quadrature with
        k+2+extra points per direction; pressure rows zero (a right-hand side
        for a solution with u = 0 on the boundary)."""
        k, h = self.k, self.h
        xq, wq = gauss(k + 2 + extra)
        P, W = _square_points(xq, wq)
        cells = self.all_cells()
        b = np.zeros(self.ndof + 1)
        for c in range(2):
            V, _ = self.eval_vel(c, P)
            X = (cells[:, None, :] + P[None, :, :]) * h
            F = f(X[..., 0], X[..., 1])[c]                  # (ncells, npts)
            loc = (F * W[None, :] * h ** 2) @ V.T            # (ncells, nloc)
            g = self.vel_global(c, cells)
            np.add.at(b, np.where(g >= 0, g, self.ndof), loc)
        return b[:-1]

    def l2_velocity_error(self, x, u, extra=2):
        """||u - u_h|| over the unit square (Gauss k+2+extra per direction)."""
        k, h = self.k, self.h
        xq, wq = gauss(k + 2 + extra)
        P, W = _square_points(xq, wq)
        cells = self.all_cells()
        X = (cells[:, None, :] + P[None, :, :]) * h
        U = u(X[..., 0], X[..., 1])
        xe = np.concatenate([x, [0.0]])
        err = 0.0
        for c in range(2):
            V, _ = self.eval_vel(c, P)
            g = self.vel_global(c, cells)
            uh = xe[np.where(g >= 0, g, self.ndof)] @ V      # (ncells, npts)
            err += np.sum((uh - U[c]) ** 2 * W[None, :]) * h ** 2
        return np.sqrt(err)


class Patches2D:
    """Vertex patches of the 2D problem and their pseudo-inverse local solves."""

    def __init__(self, S):
        self.S = S
        n, k = S.n, S.k
        self.verts = np.array([(i, j) for j in range(1, n) for i in range(1, n)], dtype=np.int64).reshape(-1, 2)
        self.colour = (self.verts[:, 0] % 2) + 2 * (self.verts[:, 1] % 2)
        self.nvel = (2 * k + 1) * (2 * k + 2)
        self.npres = (2 * k + 2) ** 2
        self._pinv = {}

    def dofs(self, v):
        S = self.S
        k, N1 = S.k, S.N1
        base = [(v[d] - 1) * (k + 1) for d in range(2)]
        out = []
        for c in range(2):
            lens = [2 * k + 2] * 2
            lens[c] = 2 * k + 1
            ext0 = N1 - 1 if c == 0 else N1
            i0, i1 = np.meshgrid(np.arange(lens[0]), np.arange(lens[1]), indexing="xy")
            out.append((S.offsets[c] + (base[0] + i0) + ext0 * (base[1] + i1)).ravel())
        i0, i1 = np.meshgrid(np.arange(2 * k + 2), np.arange(2 * k + 2), indexing="xy")
        out.append((S.offsets[2] + (base[0] + i0) + N1 * (base[1] + i1)).ravel())
        return np.concatenate(out)

    def patch_type(self, v):
        n = self.S.n
        return tuple((int(v[d] == 1), int(v[d] == n - 1)) for d in range(2))

    def pinv(self, K, v):
        key = self.patch_type(v)
        if key not in self._pinv:
            idx = self.dofs(v)
            Kj = K[idx][:, idx].toarray()
            lam, Q = np.linalg.eigh(Kj)
            keep = np.ones(len(lam), dtype=bool)
            keep[np.argmin(np.abs(lam))] = False
            self._pinv[key] = (Q[:, keep] / lam[keep]) @ Q[:, keep].T
        return self._pinv[key]


def prolongation2d(Sc, Sf):
    """Canonical embedding from Sc (n cells per direction) into Sf (2n): the
    coarse basis functions evaluated at the fine support points."""
    assert Sf.n == 2 * Sc.n and Sf.k == Sc.k
    k, H = Sf.k, Sc.h
    xg, xl = Sf.basis.dg_nodes, Sf.basis.cont_nodes
    dg_coord = (np.repeat(np.arange(Sf.n), k + 1) + np.tile(xg, Sf.n)) * Sf.h
    cont_coord = np.concatenate([(i + xl[:-1]) * Sf.h for i in range(Sf.n)] + [[1.0]])[1:-1]
    rows, cols, vals = [], [], []
    for c in range(3):
        coords = [dg_coord, dg_coord]
        kinds = ["dg", "dg"]
        if c < 2:
            coords[c] = cont_coord
            kinds[c] = "cont"
        Y, X = np.meshgrid(coords[1], coords[0], indexing="ij")
        P = np.stack([X.ravel(), Y.ravel()], axis=1)
        cell = np.clip(np.floor(P / H).astype(np.int64), 0, Sc.n - 1)
        ref = P / H - cell
        fine_idx = Sf.offsets[c] + np.arange(P.shape[0])
        V1 = [Sc.basis.values(kinds[d], ref[:, d]) for d in range(2)]
        tup = Sc.local_tuples([Sc.basis.size(kd) for kd in kinds])
        vals_c = np.array([V1[0][b0] * V1[1][b1] for (b0, b1) in tup]).T
        gidx = Sc.vel_global(c, cell) if c < 2 else Sc.pres_global(cell)
        ok = (gidx >= 0) & (np.abs(vals_c) > 0)
        rows.append(np.broadcast_to(fine_idx[:, None], gidx.shape)[ok])
        cols.append(gidx[ok])
        vals.append(vals_c[ok])
    Pm = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(Sf.ndof, Sc.ndof)).tocsr()
    Pm.sum_duplicates()
    return Pm


class Multigrid2D:
    """Levels n = n_coarse, 2 n_coarse, ..., n_fine; multiplicative sweeps over
    the 4 colours before and after the coarse correction; pseudo-inverse on
    the coarsest level."""

    def __init__(self, n_fine, k, n_coarse=1, penalty_factor=2.0):
        self.levels = []
        n = n_coarse
        while n <= n_fine:
            S = Stokes2D(n, k, penalty_factor)
            self.levels.append(dict(S=S, K=S.assemble(), patches=Patches2D(S) if n >= 2 else None))
            n *= 2
        assert self.levels[-1]["S"].n == n_fine
        self.P = [None] + [prolongation2d(self.levels[l - 1]["S"], self.levels[l]["S"])
                           for l in range(1, len(self.levels))]
        K0 = self.levels[0]["K"].toarray()
        lam, Q = np.linalg.eigh(K0)
        keep = np.ones(len(lam), dtype=bool)
        keep[np.argmin(np.abs(lam))] = False
        self.K0_pinv = (Q[:, keep] / lam[keep]) @ Q[:, keep].T

    @property
    def fine(self):
        return self.levels[-1]

    def smooth(self, l, x, b):
        lev = self.levels[l]
        K, Pt = lev["K"], lev["patches"]
        x = np.array(x, dtype=np.float64)
        for c in range(4):
            verts = Pt.verts[Pt.colour == c]
            if len(verts) == 0:
                continue
            r = b - K @ x
            dx = np.zeros_like(x)
            for v in verts:
                idx = Pt.dofs(v)
                dx[idx] += Pt.pinv(K, v) @ r[idx]
            x += dx
        return x

    def vcycle(self, b, l=None, pre=1, post=1):
        """x = P_l^{-1} b from x = 0: pre sweeps, coarse-grid correction with
        restriction P^T, post sweeps (Sec. 3)."""
        if l is None:
            l = len(self.levels) - 1
        if l == 0:
            return self.K0_pinv @ b
        x = np.zeros_like(b)
        for _ in range(pre):
            x = self.smooth(l, x, b)
        r = b - self.levels[l]["K"] @ x
        x = x + self.P[l] @ self.vcycle(self.P[l].T @ r, l - 1, pre, post)
        for _ in range(post):
            x = self.smooth(l, x, b)
        return x


def manufactured_2d(mu, sigma):
    """(u, p, f) of the Sec. 3.3 test problem in 2D as functions of (x, y)
    arrays: u = (d_y psi, -d_x psi), psi = phi(x) phi(y), p = cos(2 pi x)
    cos(2 pi y), f = -Laplace(u) + grad(p)."""
    C = 1.0 / np.sqrt(2.0 * np.pi * sigma ** 2)
    g = [np.poly1d([1.0, -2.0, 1.0, 0.0, 0.0])]        # x^2 (x-1)^2 and its derivatives
    for _ in range(3):
        g.append(np.polyder(g[-1]))

    def e_der(x, m):
        s = (x - mu) / sigma ** 2
        e = np.exp(-((x - mu) ** 2) / sigma ** 2)
        if m == 0:
            return e
        if m == 1:
            return -2.0 * s * e
        if m == 2:
            return (4.0 * s ** 2 - 2.0 / sigma ** 2) * e
        return (-8.0 * s ** 3 + 12.0 * s / sigma ** 2) * e

    def phi(x, m=0):
        return C * sum(comb(m, j) * g[j](x) * e_der(x, m - j) for j in range(m + 1))

    def u(x, y):
        return np.array([phi(x) * phi(y, 1), -phi(x, 1) * phi(y)])

    def p(x, y):
        return np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y)

    def f(x, y):
        fx = -phi(x, 2) * phi(y, 1) - phi(x) * phi(y, 3) - 2 * np.pi * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        fy = phi(x, 3) * phi(y) + phi(x, 1) * phi(y, 2) - 2 * np.pi * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y)
        return np.array([fx, fy])

    return u, p, f, phi
