"""GPU parity of stokes_apply / stokes_residual (HIP, through the C ABI)
against the oracle's element-by-element operator.

Tolerances: FP64 <= 1e-12 relative 2-norm, FP32 <= 1e-5 (per block as well:
velocity and pressure rows).  Inputs: x ~ U[-1, 1] from PCG64(seed).
"""
import numpy as np
import pytest

from gpu_common import need_gpu, announce, rel_err, block_errs
from oracle.stokes import Stokes
from paper_2410_09497_amd import StokesMG, StokesMGError
from paper_2410_09497_amd.synth import uniform_vector

pytestmark = pytest.mark.gpu

# (finest n, k): every level of the hierarchy is checked (1^3 .. n^3)
CASES = [(8, 1), (8, 2), (4, 3), (4, 4), (2, 5)]


@pytest.mark.parametrize("n,k", CASES)
def test_apply_all_levels_f64_f32(n, k):
    torch = need_gpu()
    mg = StokesMG(n, k)
    for level in range(mg.n_levels):
        nl = n >> (mg.n_levels - 1 - level)
        S = Stokes(nl, k)
        x = uniform_vector(S.ndof, seed=1000 * k + nl)
        yref = S.apply(x)
        announce("apply", f"n={nl} k={k} level={level}")
        xd = torch.from_numpy(x).cuda()
        y = mg.apply(xd, level=level).cpu().numpy()
        e, eu, ep = block_errs(S, y, yref)
        assert e <= 1e-12 and eu <= 1e-12 and ep <= 1e-12, (nl, k, e, eu, ep)
        y32 = mg.apply(xd.float(), level=level).double().cpu().numpy()
        e, eu, ep = block_errs(S, y32, yref)
        assert e <= 1e-5 and eu <= 1e-5 and ep <= 1e-5, (nl, k, e, eu, ep)


@pytest.mark.parametrize("n,k", [(8, 1), (4, 2), (2, 4)])
def test_residual(n, k):
    torch = need_gpu()
    mg = StokesMG(n, k)
    S = Stokes(n, k)
    x = uniform_vector(S.ndof, seed=5)
    b = uniform_vector(S.ndof, seed=6)
    rref = b - S.apply(x)
    announce("residual", f"n={n} k={k}")
    r = mg.residual(torch.from_numpy(b).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel_err(r, rref) <= 1e-12
    r32 = mg.residual(torch.from_numpy(b).float().cuda(), torch.from_numpy(x).float().cuda())
    assert rel_err(r32.double().cpu().numpy(), rref) <= 1e-5


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_apply_multi_tile_multi_chunk(k):
    """16^3 cells, full vector: the launch splits the level into several xy
    tiles (some ragged at k = 2, 5) and two z chunks, so the inter-tile and
    inter-chunk halos are compared with the oracle; the residual form too."""
    torch = need_gpu()
    n = 16
    mg = StokesMG(n, k, n_levels=1)
    S = Stokes(n, k)
    x = uniform_vector(S.ndof, seed=300 + k)
    b = uniform_vector(S.ndof, seed=400 + k)
    yref = S.apply(x)
    announce("apply tiles+chunks", f"n={n} k={k}")
    xd = torch.from_numpy(x).cuda()
    bd = torch.from_numpy(b).cuda()
    y = mg.apply(xd).cpu().numpy()
    e, eu, ep = block_errs(S, y, yref)
    assert e <= 1e-12 and eu <= 1e-12 and ep <= 1e-12, (k, e, eu, ep)
    y32 = mg.apply(xd.float()).double().cpu().numpy()
    e, eu, ep = block_errs(S, y32, yref)
    assert e <= 1e-5 and eu <= 1e-5 and ep <= 1e-5, (k, e, eu, ep)
    r = mg.residual(bd, xd).cpu().numpy()
    assert rel_err(r, b - yref) <= 1e-12
    r32 = mg.residual(bd.float(), xd.float()).double().cpu().numpy()
    assert rel_err(r32, b - yref) <= 1e-5


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_apply_full_size_sampled_rows(k):
    """64^3 cells (the benchmark size of every degree): rows sampled across
    the domain, including the first and last rows of every block, computed
    one by one by the oracle; the residual form too (the kernels the
    smoother and FGMRES launch at this size)."""
    torch = need_gpu()
    n = 64
    mg = StokesMG(n, k, n_levels=1)
    S = Stokes(n, k)
    x = uniform_vector(S.ndof, seed=k)
    b = uniform_vector(S.ndof, seed=50 + k)
    announce("apply full size", f"n={n} k={k}")
    xd = torch.from_numpy(x).cuda()
    y = mg.apply(xd).cpu().numpy()
    y32 = mg.apply(xd.float()).double().cpu().numpy()
    bd = torch.from_numpy(b).cuda()
    r = mg.residual(bd, xd).cpu().numpy()
    r32 = mg.residual(bd.float(), xd.float()).double().cpu().numpy()
    del bd, xd
    rng = np.random.default_rng(99)
    edges = []
    for o in list(S.offsets) + [S.ndof]:
        edges += [o - 2, o - 1, o, o + 1]
    rows = np.unique(np.clip(np.concatenate([rng.integers(0, S.ndof, 300), edges]), 0, S.ndof - 1))
    yref = S.apply_rows(x, rows)
    scale = np.abs(yref).max()
    assert np.abs(y[rows] - yref).max() <= 1e-12 * scale
    assert np.abs(y32[rows] - yref).max() <= 2e-5 * scale
    rref = b[rows] - yref
    assert np.abs(r[rows] - rref).max() <= 1e-12 * scale
    assert np.abs(r32[rows] - rref).max() <= 2e-5 * scale


def test_apply_rejects_bad_arguments():
    torch = need_gpu()
    mg = StokesMG(4, 1)
    x = torch.zeros(mg.ndof(), dtype=torch.float64, device="cuda")
    with pytest.raises(StokesMGError) as e:
        mg.apply(x, x)                      # aliasing
    assert e.value.code == -1
    with pytest.raises(ValueError):
        mg.apply(x[:-1])                    # wrong size (caught before the ABI)
    from paper_2410_09497_amd import _lib
    y = torch.zeros_like(x)
    rc = _lib.lib.stokes_apply(mg._h, 7, 0, x.data_ptr(), y.data_ptr(), None)
    assert rc == -1                        # level out of range
    rc = _lib.lib.stokes_apply(mg._h, 2, 5, x.data_ptr(), y.data_ptr(), None)
    assert rc == -1                        # dtype


def test_apply_deterministic():
    torch = need_gpu()
    mg = StokesMG(8, 2)
    x = torch.from_numpy(uniform_vector(mg.ndof(), seed=3)).cuda()
    announce("determinism n=8 k=2")
    y1 = mg.apply(x)
    y2 = mg.apply(x)
    assert torch.equal(y1, y2)
