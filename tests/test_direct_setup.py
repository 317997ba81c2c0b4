"""The Direct solver's matrices (Sec. 3.3 "Direct solver"), one per patch
type, built by the library on the host from the fast-diagonalization tables,
against the oracle's dense pseudo-inverse of the assembled patch matrix
(CPU; no device).  In the normalized variables of the patch gather,
x = (F / h, G / h^2) and t = (U, h P), the map is t = M x with
M = diag(I, h I) K_j^+ diag(h I, h^2 I), the same on every level.  The type
of the patch around vertex v is t_x + 3 t_y + 9 t_z with t_d = 1 when the
lower outer face lies on the boundary (v_d = 1), 2 for the upper one
(v_d = n - 1), 0 for neither; 27 for the patch of n = 2 (both)."""
import ctypes

import numpy as np
import pytest

from oracle.patches import Patches
from oracle.stokes import Stokes


def library_map(k, patch_type=0):
    from paper_2410_09497_amd import load_library
    L = load_library()
    h = ctypes.c_void_p()
    cfg = L.Config(8, k, 1, 2.0, 1e-10, 50)
    assert L.lib.stokesmg_create(ctypes.byref(cfg), ctypes.byref(h)) == L.OK
    d = ctypes.c_int64()
    assert L.lib.mlp_dims(h, ctypes.byref(d), None) == L.OK
    M = np.empty((d.value, d.value))
    assert L.lib.stokesmg_direct_matrix(h, patch_type, M.ctypes.data) == L.OK
    L.lib.stokesmg_destroy(h)
    return M


def type_index(P, v):
    t = [lo + 2 * hi for lo, hi in P.patch_type(v)]
    return 27 if t == [3, 3, 3] else t[0] + 3 * t[1] + 9 * t[2]


def oracle_maps(n, k, vertices):
    S = Stokes(n, k)
    K = S.assemble()
    P = Patches(S)
    nu = 3 * P.nvel
    din = np.concatenate([np.full(nu, S.h), np.full(P.npres, S.h ** 2)])
    dout = np.concatenate([np.ones(nu), np.full(P.npres, S.h)])
    return {type_index(P, np.array(v)): dout[:, None] * P.pinv(K, np.array(v)) * din[None, :] for v in vertices}


@pytest.mark.parametrize("k", [1, 2])
def test_direct_map_equals_oracle_pseudo_inverse(k):
    M = library_map(k)
    for n in (4, 6):                               # two levels: the normalized map is level independent
        Mo = oracle_maps(n, k, [(2, 2, 2)])[0]     # interior vertex: its cells touch no boundary face
        assert np.abs(M - Mo).max() <= 1e-9 * np.abs(Mo).max(), n


def test_direct_maps_of_every_boundary_type_k1():
    # n = 4: vertex coordinates 1, 2, 3 give t_d = 1, 0, 2; all 27 types
    verts = [(a, b, c) for c in (1, 2, 3) for b in (1, 2, 3) for a in (1, 2, 3)]
    Mo = oracle_maps(4, 1, verts)
    assert sorted(Mo) == list(range(27))
    for t, Mt in Mo.items():
        M = library_map(1, t)
        assert np.abs(M - Mt).max() <= 1e-9 * np.abs(Mt).max(), t
    # the types differ from each other (the boundary faces enter A)
    assert np.abs(Mo[1] - Mo[0]).max() > 1e-3 * np.abs(Mo[0]).max()
    assert np.abs(Mo[2] - Mo[1]).max() > 1e-3 * np.abs(Mo[0]).max()
    # n = 2: the single patch, both faces on the boundary in every direction
    M2 = oracle_maps(2, 1, [(1, 1, 1)])
    assert list(M2) == [27]
    M = library_map(1, 27)
    assert np.abs(M - M2[27]).max() <= 1e-9 * np.abs(M2[27]).max()


def test_direct_maps_of_boundary_types_k2_second_level():
    # a face, an edge and a corner type on the 6^3 mesh (vertex 5 = n - 1)
    Mo = oracle_maps(6, 2, [(1, 2, 2), (3, 5, 3), (1, 5, 1)])
    assert sorted(Mo) == [1, 6, 16]
    for t, Mt in Mo.items():
        M = library_map(2, t)
        assert np.abs(M - Mt).max() <= 1e-9 * np.abs(Mt).max(), t


def test_direct_matrix_rejects_bad_type():
    from paper_2410_09497_amd import load_library
    L = load_library()
    h = ctypes.c_void_p()
    cfg = L.Config(4, 1, 1, 2.0, 1e-10, 50)
    assert L.lib.stokesmg_create(ctypes.byref(cfg), ctypes.byref(h)) == L.OK
    M = np.empty((208, 208))
    assert L.lib.stokesmg_direct_matrix(h, 28, M.ctypes.data) == L.EINVAL
    assert L.lib.stokesmg_direct_matrix(h, -1, M.ctypes.data) == L.EINVAL
    L.lib.stokesmg_destroy(h)


def test_direct_matrix_rejects_high_degree():
    from paper_2410_09497_amd import load_library
    L = load_library()
    h = ctypes.c_void_p()
    cfg = L.Config(4, 4, 1, 2.0, 1e-10, 50)
    assert L.lib.stokesmg_create(ctypes.byref(cfg), ctypes.byref(h)) == L.OK
    M = np.empty(1)
    assert L.lib.stokesmg_direct_matrix(h, 0, M.ctypes.data) == L.EUNSUPPORTED
    L.lib.stokesmg_destroy(h)
