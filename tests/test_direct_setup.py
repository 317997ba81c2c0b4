"""The Direct solver's matrix (Sec. 3.3 "Direct solver", interior patches),
built by the library on the host from the fast-diagonalization tables,
against the oracle's dense pseudo-inverse of the assembled patch matrix
(CPU; no device).  In the normalized variables of the patch gather,
x = (F / h, G / h^2) and t = (U, h P), the map is t = M x with
M = diag(I, h I) K_j^+ diag(h I, h^2 I), the same on every level."""
import ctypes

import numpy as np
import pytest

from oracle.patches import Patches
from oracle.stokes import Stokes


def library_map(k):
    from paper_2410_09497_amd import load_library
    L = load_library()
    h = ctypes.c_void_p()
    cfg = L.Config(8, k, 1, 2.0, 1e-10, 50)
    assert L.lib.stokesmg_create(ctypes.byref(cfg), ctypes.byref(h)) == L.OK
    d = ctypes.c_int64()
    assert L.lib.mlp_dims(h, ctypes.byref(d), None) == L.OK
    M = np.empty((d.value, d.value))
    assert L.lib.stokesmg_direct_matrix(h, M.ctypes.data) == L.OK
    L.lib.stokesmg_destroy(h)
    return M


def oracle_map(n, k):
    S = Stokes(n, k)
    K = S.assemble()
    P = Patches(S)
    v = np.array([2, 2, 2])                       # interior vertex: its cells touch no boundary face
    assert all(t == (0, 0) for t in P.patch_type(v))
    Kp = P.pinv(K, v)
    nu = 3 * P.nvel
    din = np.concatenate([np.full(nu, S.h), np.full(P.npres, S.h ** 2)])
    dout = np.concatenate([np.ones(nu), np.full(P.npres, S.h)])
    return dout[:, None] * Kp * din[None, :]


@pytest.mark.parametrize("k", [1, 2])
def test_direct_map_equals_oracle_pseudo_inverse(k):
    M = library_map(k)
    for n in (4, 6):                               # two levels: the normalized map is level independent
        Mo = oracle_map(n, k)
        assert np.abs(M - Mo).max() <= 1e-9 * np.abs(Mo).max(), n


def test_direct_matrix_rejects_high_degree():
    from paper_2410_09497_amd import load_library
    L = load_library()
    h = ctypes.c_void_p()
    cfg = L.Config(4, 4, 1, 2.0, 1e-10, 50)
    assert L.lib.stokesmg_create(ctypes.byref(cfg), ctypes.byref(h)) == L.OK
    M = np.empty(1)
    assert L.lib.stokesmg_direct_matrix(h, M.ctypes.data) == L.EUNSUPPORTED
    L.lib.stokesmg_destroy(h)
