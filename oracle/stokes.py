"""The discrete Stokes problem of Sec. 2, built from its plain definition
(oracle; test infrastructure, float64 throughout).

Problem (Eq. model): -Laplace(u) + grad(p) = f, div(u) = 0 on the unit cube,
discretized on a uniform mesh of n^3 cubes (Sec. 2.1) with RT_k velocity
(normal component continuous; u.n = 0 on the boundary is built into the space,
so the boundary normal nodes are eliminated) and discontinuous Q_k pressure.

Operator.  Every matrix here is assembled element by element from full 3D
tensor Gauss quadrature with k+2 points per direction in cells and on faces,
which integrates every term exactly:

* cell term (grad u, grad v) of Eq. bilinear,
* interior faces: gamma [u].[v] - {{d_n u}}.[v] - [u].{{d_n v}}; this is
  Eq. bilinear's 4 gamma {{u (x) n}}:{{v (x) n}} - 2 <{{grad u}}, {{v (x) n}}>
  - 2 <{{grad v}}, {{u (x) n}}> after substituting {{u (x) n}} = 1/2 [u] (x) n,
* boundary faces: 2 gamma <u, v> - <d_n u, v> - <u, d_n v> (Eq. bilinear),
* penalty gamma = penalty_factor (k+1)^2 / h, penalty_factor = 2,
* divergence block B_{PX} = -(psi_P, div phi_X) (Eq. weak_form, written with
  the symmetric sign convention of Eq. block_A, so that the system matrix is
  K = [[A, B^T], [B, 0]] and B^T p represents (grad p, v)).

DoF layout (the vector the library also uses, a specification each side
implements on its own): [u_x | u_y | u_z | p].  Component c is a lexicographic
grid, x fastest; in its own direction c the index is the interior continuous
node g-1 (g = 1 .. N1-1, N1 = n (k+1)), in the other directions the
discontinuous index cell*(k+1) + Gauss index.  p is the N1^3 grid of
discontinuous indices.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fe1d import Basis1D, gauss


def _tensor_points(x1d, w1d):
    """3D tensor points (x fastest) and weights on the unit cube."""
    n = len(x1d)
    P = np.zeros((n ** 3, 3))
    W = np.zeros(n ** 3)
    q = 0
    for c in range(n):
        for b in range(n):
            for a in range(n):
                P[q] = (x1d[a], x1d[b], x1d[c])
                W[q] = w1d[a] * w1d[b] * w1d[c]
                q += 1
    return P, W


def _face_points(d, t1d, w1d, coord):
    """Points on the reference face x_d = coord (tensor rule in the two
    tangential directions), and their weights."""
    tang = [e for e in range(3) if e != d]
    n = len(t1d)
    P = np.zeros((n * n, 3))
    W = np.zeros(n * n)
    q = 0
    for b in range(n):
        for a in range(n):
            P[q, tang[0]] = t1d[a]
            P[q, tang[1]] = t1d[b]
            P[q, d] = coord
            W[q] = w1d[a] * w1d[b]
            q += 1
    return P, W


class Stokes:
    """Discrete Stokes operator on n^3 cells with RT_k x DG Q_k."""

    def __init__(self, n, k, penalty_factor=2.0):
        if n < 1 or k < 1:
            raise ValueError("need n >= 1 and k >= 1")
        self.n, self.k = n, k
        self.h = 1.0 / n
        self.N1 = n * (k + 1)
        self.nc = (self.N1 - 1) * self.N1 * self.N1
        self.npres = self.N1 ** 3
        self.ndof = 3 * self.nc + self.npres
        self.offsets = (0, self.nc, 2 * self.nc, 3 * self.nc)
        self.gamma = penalty_factor * (k + 1) ** 2 / self.h
        self.basis = Basis1D(k)
        self._local = None

    # ------------------------------------------------------------------ layout
    def vel_sizes(self, c):
        s = [self.k + 1] * 3
        s[c] = self.k + 2
        return s

    def local_tuples(self, sizes):
        """Local basis tuples (b0, b1, b2), b0 fastest."""
        return [(b0, b1, b2) for b2 in range(sizes[2]) for b1 in range(sizes[1]) for b0 in range(sizes[0])]

    def vel_global(self, c, cells):
        """Global indices (ncells, nloc) of component c's local basis functions
        on the given cells; -1 marks an eliminated boundary normal node."""
        k, N1 = self.k, self.N1
        cells = np.atleast_2d(cells)
        tup = np.array(self.local_tuples(self.vel_sizes(c)))  # (nloc, 3)
        idx = []
        ext = []
        valid = np.ones((cells.shape[0], tup.shape[0]), dtype=bool)
        for d in range(3):
            pos = cells[:, d:d + 1] * (k + 1) + tup[None, :, d]
            if d == c:
                valid &= (pos > 0) & (pos < N1)
                idx.append(pos - 1)
                ext.append(N1 - 1)
            else:
                idx.append(pos)
                ext.append(N1)
        g = self.offsets[c] + idx[0] + ext[0] * (idx[1] + ext[1] * idx[2])
        return np.where(valid, g, -1)

    def pres_global(self, cells):
        k, N1 = self.k, self.N1
        cells = np.atleast_2d(cells)
        tup = np.array(self.local_tuples([k + 1] * 3))
        pos = [cells[:, d:d + 1] * (k + 1) + tup[None, :, d] for d in range(3)]
        return self.offsets[3] + pos[0] + N1 * (pos[1] + N1 * pos[2])

    def all_cells(self):
        n = self.n
        i0, i1, i2 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        return np.stack([i0.ravel(), i1.ravel(), i2.ravel()], axis=1)

    # ------------------------------------------------------- basis evaluation
    def eval_vel(self, c, P):
        """Values (nloc, npts) and reference gradients (3, nloc, npts) of the
        component-c velocity basis at reference points P (npts, 3)."""
        kinds = ["dg"] * 3
        kinds[c] = "cont"
        V1 = [self.basis.values(kinds[d], P[:, d]) for d in range(3)]
        D1 = [self.basis.derivatives(kinds[d], P[:, d]) for d in range(3)]
        tup = self.local_tuples(self.vel_sizes(c))
        val = np.array([V1[0][b0] * V1[1][b1] * V1[2][b2] for (b0, b1, b2) in tup])
        grad = np.zeros((3,) + val.shape)
        for i, (b0, b1, b2) in enumerate(tup):
            grad[0, i] = D1[0][b0] * V1[1][b1] * V1[2][b2]
            grad[1, i] = V1[0][b0] * D1[1][b1] * V1[2][b2]
            grad[2, i] = V1[0][b0] * V1[1][b1] * D1[2][b2]
        return val, grad

    def eval_pres(self, P):
        V1 = [self.basis.values("dg", P[:, d]) for d in range(3)]
        tup = self.local_tuples([self.k + 1] * 3)
        return np.array([V1[0][b0] * V1[1][b1] * V1[2][b2] for (b0, b1, b2) in tup])

    # ---------------------------------------------------------- local matrices
    def local_matrices(self):
        """Cell, interior-face and boundary-face matrices (identical for every
        cell / face of one orientation on the uniform mesh)."""
        if self._local is not None:
            return self._local
        k, h, gam = self.k, self.h, self.gamma
        xq, wq = gauss(k + 2)
        P, W = _tensor_points(xq, wq)
        W = W * h ** 3
        Q = self.eval_pres(P)
        cell_A, cell_B = [], []
        for c in range(3):
            V, G = self.eval_vel(c, P)
            G = G / h
            cell_A.append(sum(G[e] @ (W[:, None] * G[e].T) for e in range(3)))
            cell_B.append(-(Q @ (W[:, None] * G[c].T)))
        face = {}
        bface = {}
        for d in range(3):
            Pm, Wf = _face_points(d, xq, wq, 1.0)   # on the minus cell: x_d = 1
            Pp, _ = _face_points(d, xq, wq, 0.0)    # on the plus cell:  x_d = 0
            Wf = Wf * h ** 2
            for c in range(3):
                Vm, Gm = self.eval_vel(c, Pm)
                Vp, Gp = self.eval_vel(c, Pp)
                Nm, Np = Gm[d] / h, Gp[d] / h      # derivative along n^- = +e_d
                J = np.concatenate([Vm, -Vp])      # jump [u] = u^- - u^+
                Av = 0.5 * np.concatenate([Nm, Np])
                JW = J * Wf[None, :]
                face[(d, c)] = gam * JW @ J.T - JW @ Av.T - (Av * Wf[None, :]) @ J.T
                for side in (0, 1):
                    Pb, _ = _face_points(d, xq, wq, float(side))
                    Vb, Gb = self.eval_vel(c, Pb)
                    Nb = (1.0 if side == 1 else -1.0) * Gb[d] / h   # outward normal derivative
                    VW = Vb * Wf[None, :]
                    bface[(d, side, c)] = 2.0 * gam * VW @ Vb.T - VW @ Nb.T - (Nb * Wf[None, :]) @ Vb.T
        # Products of Gauss-point Lagrange polynomials integrated exactly are
        # orthogonal, so many entries are exactly zero mathematically and come
        # out as rounding residue (relative size <= 1e-15, while every true
        # entry is >= 1e-7 relative for k <= 5).  Residue below 1e-12 of the
        # block's largest entry is set to zero so the sparse pattern is the
        # true one.
        def clean(M):
            M = M.copy()
            M[np.abs(M) < 1e-12 * np.abs(M).max()] = 0.0
            return M

        self._local = dict(cell_A=[clean(M) for M in cell_A], cell_B=[clean(M) for M in cell_B],
                           face={key: clean(M) for key, M in face.items()},
                           bface={key: clean(M) for key, M in bface.items()})
        return self._local

    # ------------------------------------------------------- block enumeration
    def blocks(self):
        """Yield (row_idx (m, r), col_idx (m, c), M (r, c)) for every local
        block of K; rows/cols of -1 are eliminated DoFs."""
        L = self.local_matrices()
        n = self.n
        cells = self.all_cells()
        P = self.pres_global(cells)
        for c in range(3):
            R = self.vel_global(c, cells)
            yield R, R, L["cell_A"][c]
            yield P, R, L["cell_B"][c]
            yield R, P, L["cell_B"][c].T
        for d in range(3):
            e = np.zeros(3, dtype=int)
            e[d] = 1
            minus = cells[cells[:, d] < n - 1]
            plus = minus + e
            lo = cells[cells[:, d] == 0]
            hi = cells[cells[:, d] == n - 1]
            for c in range(3):
                R = np.concatenate([self.vel_global(c, minus), self.vel_global(c, plus)], axis=1)
                if R.shape[0]:
                    yield R, R, L["face"][(d, c)]
                Rl = self.vel_global(c, lo)
                yield Rl, Rl, L["bface"][(d, 0, c)]
                Rh = self.vel_global(c, hi)
                yield Rh, Rh, L["bface"][(d, 1, c)]

    # ------------------------------------------------------------ assembly
    def assemble(self):
        """Global sparse K = [[A, B^T], [B, 0]] in CSR (sums of local blocks)."""
        rows, cols, vals = [], [], []
        for R, C, M in self.blocks():
            nzr, nzc = np.nonzero(M)
            Rr = R[:, nzr]
            Cc = C[:, nzc]
            V = np.broadcast_to(M[nzr, nzc], Rr.shape)
            ok = (Rr >= 0) & (Cc >= 0)
            rows.append(Rr[ok])
            cols.append(Cc[ok])
            vals.append(V[ok])
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        K = sp.coo_matrix((vals, (rows, cols)), shape=(self.ndof, self.ndof)).tocsr()
        K.sum_duplicates()
        return K

    def apply(self, x):
        """y = K x by local matrices (gather, multiply, scatter-add); no
        global matrix is formed, so this also runs at large n."""
        x = np.asarray(x, dtype=np.float64)
        xe = np.concatenate([x, [0.0]])          # index -1 reads zero
        y = np.zeros(self.ndof)
        for R, C, M in self.blocks():
            if R.shape[0] == 0:
                continue
            loc = xe[C] @ M.T
            ok = R >= 0
            y += np.bincount(R[ok], weights=loc[ok], minlength=self.ndof)
        return y

    def apply_rows(self, x, rows):
        """(K x)[rows] for a few rows, from the local blocks touching them."""
        rows = np.asarray(rows)
        want = np.full(self.ndof + 1, -1, dtype=np.int64)
        want[rows] = np.arange(len(rows))
        xe = np.concatenate([np.asarray(x, dtype=np.float64), [0.0]])
        out = np.zeros(len(rows))
        for R, C, M in self.blocks():
            if R.shape[0] == 0:
                continue
            hit = (want[R] >= 0).any(axis=1)
            if not hit.any():
                continue
            Rh, Ch = R[hit], C[hit]
            loc = xe[Ch] @ M.T
            w = want[Rh]
            ok = w >= 0
            out += np.bincount(w[ok], weights=loc[ok], minlength=len(rows))
        return out

    # ----------------------------------------------------- pressure helpers
    def pressure_weights(self):
        """Integral of each pressure basis function: h^3 w_a w_b w_c."""
        w1 = np.tile(self.basis.dg_weights, self.n) * self.h     # per 1D index
        return np.einsum("k,j,i->kji", w1, w1, w1).ravel()       # x fastest

    def pressure_mean(self, x):
        """Integral mean of p_h over the unit cube."""
        return float(self.pressure_weights() @ x[self.offsets[3]:])

    def normalize_pressure(self, x):
        x = np.array(x, dtype=np.float64)
        x[self.offsets[3]:] -= self.pressure_mean(x)
        return x

    # --------------------------------------------------- right-hand sides
    def rhs(self, f, g=None):
        """F_X = (f, phi_X) + sum over boundary faces of
        2 gamma <g, phi_X> - <g, d_n phi_X> (the Nitsche terms that the
        boundary part of Eq. bilinear produces for tangential data g); the
        pressure rows are zero.  f, g: callables (x, y, z) -> (3, ...)."""
        k, h, n = self.k, self.h, self.n
        xq, wq = gauss(k + 2)
        P, W = _tensor_points(xq, wq)
        W = W * h ** 3
        cells = self.all_cells()
        X = (cells[:, None, :] + P[None, :, :]) * h
        fv = np.asarray(f(X[..., 0], X[..., 1], X[..., 2]))
        b = np.zeros(self.ndof)
        for c in range(3):
            V, _ = self.eval_vel(c, P)
            loc = (fv[c] * W[None, :]) @ V.T
            R = self.vel_global(c, cells)
            ok = R >= 0
            b += np.bincount(R[ok], weights=loc[ok], minlength=self.ndof)
        if g is None:
            return b
        for d in range(3):
            for side in (0, 1):
                Pb, Wf = _face_points(d, xq, wq, float(side))
                Wf = Wf * h ** 2
                bc = cells[cells[:, d] == (0 if side == 0 else n - 1)]
                X = (bc[:, None, :] + Pb[None, :, :]) * h
                gv = np.asarray(g(X[..., 0], X[..., 1], X[..., 2]))
                for c in range(3):
                    Vb, Gb = self.eval_vel(c, Pb)
                    Nb = (1.0 if side == 1 else -1.0) * Gb[d] / h
                    gw = gv[c] * Wf[None, :]
                    loc = 2.0 * self.gamma * gw @ Vb.T - gw @ Nb.T
                    R = self.vel_global(c, bc)
                    ok = R >= 0
                    b += np.bincount(R[ok], weights=loc[ok], minlength=self.ndof)
        return b

    # ------------------------------------------------------------- norms
    def l2_errors(self, x, u_exact, p_exact, extra=1):
        """L2 errors ||u - u_h||, ||p - p_h|| with Gauss (k+2+extra)^3 per cell;
        both pressures are taken with zero integral mean."""
        k, h = self.k, self.h
        xq, wq = gauss(k + 2 + extra)
        P, W = _tensor_points(xq, wq)
        W = W * h ** 3
        cells = self.all_cells()
        X = (cells[:, None, :] + P[None, :, :]) * h
        ue = np.asarray(u_exact(X[..., 0], X[..., 1], X[..., 2]))
        xe = np.concatenate([x, [0.0]])
        eu = 0.0
        for c in range(3):
            V, _ = self.eval_vel(c, P)
            uh = xe[self.vel_global(c, cells)] @ V
            eu += float(((uh - ue[c]) ** 2 * W[None, :]).sum())
        pe = np.asarray(p_exact(X[..., 0], X[..., 1], X[..., 2]))
        pe = pe - (pe * W[None, :]).sum()          # exact pressure mean (volume 1)
        xn = self.normalize_pressure(x)
        Q = self.eval_pres(P)
        ph = xn[self.pres_global(cells)] @ Q
        ep = float(((ph - pe) ** 2 * W[None, :]).sum())
        return np.sqrt(eu), np.sqrt(ep)

    # ------------------------------------------------------ interpolation
    def interpolate(self, u_exact, p_exact):
        """Nodal interpolant: every coefficient is the function's component
        at the DoF's support point."""
        k, h, N1 = self.k, self.h, self.N1
        xg = self.basis.dg_nodes
        xl = self.basis.cont_nodes
        dg_coord = (np.repeat(np.arange(self.n), k + 1) + np.tile(xg, self.n)) * h          # N1 points
        cont_coord = np.concatenate([(i + xl[:-1]) * h for i in range(self.n)] + [[1.0]])  # N1+1 nodes
        cont_int = cont_coord[1:-1]
        x = np.zeros(self.ndof)
        for c in range(3):
            coords = [dg_coord] * 3
            coords[c] = cont_int
            Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
            x[self.offsets[c]:self.offsets[c] + self.nc] = np.asarray(u_exact(X, Y, Z))[c].ravel()
        Z, Y, X = np.meshgrid(dg_coord, dg_coord, dg_coord, indexing="ij")
        x[self.offsets[3]:] = np.asarray(p_exact(X, Y, Z)).ravel()
        return x

    # ------------------------------------------------------- direct solve
    def direct_solve(self, b, K=None, tol=1e-14, maxit=2000):
        """Solution of K x = b with zero integral mean pressure.

        The block elimination of K = [[A, B^T], [B, 0]]: A is block diagonal
        over the three velocity components (the cell gradient and the face
        terms act componentwise), each block is factored by sparse LU, and
        the pressure solves the Schur complement system
        B A^{-1} B^T p = B A^{-1} F - G by conjugate gradients on the
        complement of the constant vector (constants span the kernel of B^T);
        then u = A^{-1}(F - B^T p), and p is shifted to zero integral mean.
        CG runs to a relative residual of ``tol``, so the result is the exact
        solution up to that tolerance.
        """
        if K is None:
            K = self.assemble()
        K = K.tocsr()
        o = self.offsets
        b = np.asarray(b, dtype=np.float64)
        lus = [spla.splu(K[o[c]:o[c + 1], o[c]:o[c + 1]].tocsc()) for c in range(3)]
        Bm = K[o[3]:, :o[3]].tocsr()
        BT = K[:o[3], o[3]:].tocsr()

        def Ainv(v):
            return np.concatenate([lus[c].solve(v[o[c]:o[c + 1]]) for c in range(3)])

        def proj(q):
            return q - q.mean()

        def S(q):
            return proj(Bm @ Ainv(BT @ q))

        F, G = b[:o[3]], b[o[3]:]
        rhs = proj(Bm @ Ainv(F) - G)
        p = np.zeros(self.npres)
        r = rhs.copy()
        d = r.copy()
        rr = r @ r
        nrm0 = np.sqrt(rr)
        if nrm0 > 0:
            for _ in range(maxit):
                Sd = S(d)
                alpha = rr / (d @ Sd)
                p += alpha * d
                r -= alpha * Sd
                rr_new = r @ r
                if np.sqrt(rr_new) <= tol * nrm0:
                    break
                d = r + (rr_new / rr) * d
                rr = rr_new
        u = Ainv(F - BT @ p)
        return self.normalize_pressure(np.concatenate([u, p]))
