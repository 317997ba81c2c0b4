"""Vertex patches and local solvers (oracle; test infrastructure, float64).

Sec. 3.1: one patch per interior vertex; in 3D a patch holds the 8 cells
around its vertex.  The local space X_j holds the functions supported inside
the patch: every tangential velocity and pressure DoF of the 8 cells and the
normal velocity DoFs on faces interior to the patch; the normal nodes on the
patch boundary are not part of X_j (caption of Fig. smoother).

In the DoF layout of ``stokes`` a patch around vertex (v0, v1, v2),
1 <= v_d <= n-1, is a box of every component's index grid starting at
base_d = (v_d - 1)(k+1): 2k+1 indices in a component's own (continuous)
direction and 2k+2 in each discontinuous direction and for the pressure.
The patch-local vector is [U_x | U_y | U_z | P], each a lexicographic
sub-grid with x fastest.

Colours (Fig. patch_coloring): 2^3 colours, colour of vertex v =
(v0 mod 2) + 2 (v1 mod 2) + 4 (v2 mod 2); patches of one colour have disjoint
DoF sets.

Local solver (Sec. 3.1 and the "Direct solver" of Sec. 3.3): the patch matrix
is the Galerkin restriction K_j = K[X_j, X_j] (the local problem defining
P_{l,j}), and the correction is K_j^+ R_j r with the pseudo-inverse that
omits the one zero eigenvalue (constant patch pressure).

Two routes to K_j^+ R_j r: ``solver="pinv"`` (default) forms the dense
pseudo-inverse by a symmetric eigendecomposition; ``solver="bordered"``
solves the system bordered by the kernel vector c (constant patch
pressure), [[K_j, c], [c^T, 0]] (x, l) = (r, 0), by an LU factorization:
since c^T K_j = 0, l = c.r / c.c and K_j x = r - l c with c.x = 0, which is
K_j^+ r.  The second route serves the large patches of degrees 4 and 5
(3700 and 6480 unknowns); both are compared in the tests.
"""
import numpy as np
import scipy.linalg as sla


class Patches:
    def __init__(self, S, solver="pinv"):
        assert solver in ("pinv", "bordered")
        self.S = S
        self.solver = solver
        self._lu = {}
        n, k = S.n, S.k
        self.verts = np.array([(i, j, l) for l in range(1, n) for j in range(1, n) for i in range(1, n)],
                              dtype=np.int64).reshape(-1, 3)
        self.colour = (self.verts[:, 0] % 2) + 2 * (self.verts[:, 1] % 2) + 4 * (self.verts[:, 2] % 2)
        self.nvel = (2 * k + 1) * (2 * k + 2) ** 2
        self.npres = (2 * k + 2) ** 3
        self.size = 3 * self.nvel + self.npres
        self._pinv = {}

    def dofs(self, v):
        """Global indices of X_j for vertex v, in patch-local order."""
        S = self.S
        k, N1 = S.k, S.N1
        base = [(v[d] - 1) * (k + 1) for d in range(3)]
        out = []
        for c in range(3):
            lens = [2 * k + 2] * 3
            lens[c] = 2 * k + 1
            ext = [N1] * 3
            ext[c] = N1 - 1
            i2, i1, i0 = np.meshgrid(np.arange(lens[2]) + base[2], np.arange(lens[1]) + base[1],
                                     np.arange(lens[0]) + base[0], indexing="ij")
            out.append((S.offsets[c] + i0 + ext[0] * (i1 + ext[1] * i2)).ravel())
        m = 2 * k + 2
        i2, i1, i0 = np.meshgrid(np.arange(m) + base[2], np.arange(m) + base[1], np.arange(m) + base[0],
                                 indexing="ij")
        out.append((S.offsets[3] + i0 + N1 * (i1 + N1 * i2)).ravel())
        return np.concatenate(out)

    def patch_type(self, v):
        """Which outer patch faces are domain boundaries, per direction:
        (lower is boundary, upper is boundary)."""
        n = self.S.n
        return tuple((int(v[d] == 1), int(v[d] == n - 1)) for d in range(3))

    def local_matrix(self, K, v):
        idx = self.dofs(v)
        return K[idx][:, idx].toarray()

    def pinv(self, K, v):
        """Pseudo-inverse of K_j dropping the single zero eigenvalue.  Patches
        with the same boundary type have identical matrices; cached by type."""
        key = self.patch_type(v)
        if key not in self._pinv:
            Kj = self.local_matrix(K, v)
            lam, Q = np.linalg.eigh(Kj)
            drop = np.argmin(np.abs(lam))
            keep = np.ones(len(lam), dtype=bool)
            keep[drop] = False
            self._pinv[key] = (Q[:, keep] / lam[keep]) @ Q[:, keep].T
        return self._pinv[key]

    def bordered_lu(self, K, v):
        """LU factors (LAPACK, partial pivoting) of K_j bordered by the
        constant-pressure vector, cached by patch type like the
        pseudo-inverse."""
        key = self.patch_type(v)
        if key not in self._lu:
            m = self.size
            Kb = np.zeros((m + 1, m + 1))
            Kb[:m, :m] = self.local_matrix(K, v)
            Kb[3 * self.nvel:m, m] = 1.0
            Kb[m, 3 * self.nvel:m] = 1.0
            self._lu[key] = sla.lu_factor(Kb, overwrite_a=True, check_finite=False)
        return self._lu[key]

    def local_solve(self, K, v, rj):
        if self.solver == "pinv":
            return self.pinv(K, v) @ rj
        return sla.lu_solve(self.bordered_lu(K, v), np.concatenate([rj, [0.0]]), check_finite=False)[:-1]


def schur_local_solve(Kj, nvel, rj, tol=1e-15, maxit=10000):
    """The Schur-complement route of Sec. 3.2 with dense matrices:
    S = B A^{-1} B^T; solve S P = B A^{-1} F - G' by CG on mean-zero vectors
    (G' = G - mean(G), the part of G in the range of B), then
    U = A^{-1}(F - B^T P).  Equals K_j^+ (F, G)."""
    A = Kj[:nvel, :nvel]
    B = Kj[nvel:, :nvel]
    F, G = rj[:nvel], rj[nvel:]
    G = G - G.mean()
    Ainv_F = np.linalg.solve(A, F)
    rhs = B @ Ainv_F - G
    rhs -= rhs.mean()
    Smat = B @ np.linalg.solve(A, B.T)
    P = np.zeros(len(G))
    r = rhs.copy()
    d = r.copy()
    rr = r @ r
    r0 = np.sqrt(rr)
    for _ in range(maxit):
        if r0 == 0 or np.sqrt(rr) <= tol * r0:
            break
        Sd = Smat @ d
        Sd -= Sd.mean()
        a = rr / (d @ Sd)
        P += a * d
        r -= a * Sd
        rr_new = r @ r
        d = r + (rr_new / rr) * d
        rr = rr_new
    P -= P.mean()
    U = np.linalg.solve(A, F - B.T @ P)
    return np.concatenate([U, P])
