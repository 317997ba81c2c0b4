"""GPU parity of patch_smooth (Alg. 2 with Schur/fast-diagonalization local
solves, HIP) against the oracle's colourized smoother with pseudo-inverse
local solves (the "Direct solver" of Sec. 3.3).  With a tight local CG
tolerance the two coincide: FP64 <= 1e-10 relative.  FP32 (local CG to
1e-6): <= 1e-4 relative."""
import numpy as np
import pytest

import manufactured as mf
from gpu_common import need_gpu, announce, rel_err
from oracle.mg import Multigrid
from paper_2410_09497_amd import StokesMG
from paper_2410_09497_amd.synth import uniform_vector

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,k", [(2, 1), (4, 1), (8, 1), (2, 2), (4, 2), (4, 3)])
def test_one_sweep_f64(n, k):
    torch = need_gpu()
    mg_o = Multigrid(n, k, n_coarse=n)
    S = mg_o.fine["S"]
    x0 = uniform_vector(S.ndof, seed=10 + n + k)
    b = uniform_vector(S.ndof, seed=20 + n + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.smooth(0, x0, b)
    announce("patch_smooth f64", f"n={n} k={k}")
    mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-14, cg_max_it=500)
    x = torch.from_numpy(x0).cuda()
    mg.smooth(x, torch.from_numpy(b).cuda())
    its, solves = mg.cg_stats()
    assert solves == (n - 1) ** 3
    e = rel_err(x.cpu().numpy(), xref)
    assert e <= 1e-10, (n, k, e, its / max(solves, 1))


def test_single_patch_solves_exactly():
    """n = 2: one patch holds every unknown; one sweep from 0 is the solve."""
    torch = need_gpu()
    n, k = 2, 2
    mg_o = Multigrid(n, k)
    S, K = mg_o.fine["S"], mg_o.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-14, cg_max_it=500)
    announce("single patch exact")
    x = torch.zeros(S.ndof, dtype=torch.float64, device="cuda")
    mg.smooth(x, torch.from_numpy(b).cuda())
    xs = S.normalize_pressure(x.cpu().numpy())
    assert np.abs(xs - S.direct_solve(b, K)).max() <= 1e-10


@pytest.mark.parametrize("n,k", [(4, 1), (4, 2)])
def test_one_sweep_f32(n, k):
    torch = need_gpu()
    mg_o = Multigrid(n, k, n_coarse=n)
    S = mg_o.fine["S"]
    x0 = uniform_vector(S.ndof, seed=3)
    b = uniform_vector(S.ndof, seed=4)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.smooth(0, x0, b)
    announce("patch_smooth f32", f"n={n} k={k}")
    mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-6, cg_max_it=200)
    x = torch.from_numpy(x0).float().cuda()
    mg.smooth(x, torch.from_numpy(b).float().cuda())
    assert rel_err(x.double().cpu().numpy(), xref) <= 1e-4


def test_smoother_deterministic():
    torch = need_gpu()
    n, k = 8, 2
    mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-8, cg_max_it=100)
    x0 = torch.from_numpy(uniform_vector(mg.ndof(), seed=1)).cuda()
    b = torch.from_numpy(uniform_vector(mg.ndof(), seed=2)).cuda()
    announce("smoother determinism")
    x1 = x0.clone()
    x2 = x0.clone()
    mg.smooth(x1, b)
    mg.smooth(x2, b)
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("n,k", [(2, 4), (4, 4), (2, 5), (4, 5)])
def test_one_sweep_high_degree(n, k):
    """Degrees 4 and 5 (patches of 3700 and 6480 unknowns, 86 KB and 150 KB
    of LDS per workgroup in FP64): one sweep against the oracle, whose patch
    pseudo-inverse goes through the bordered sparse LU at these sizes.
    n = 2 is the single-patch exact solve; FP32 at n = 4 as well."""
    torch = need_gpu()
    mg_o = Multigrid(n, k, n_coarse=n, local_solver="bordered")
    S = mg_o.fine["S"]
    x0 = uniform_vector(S.ndof, seed=30 + n + k)
    b = uniform_vector(S.ndof, seed=40 + n + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.smooth(0, x0, b)
    announce("patch_smooth f64", f"n={n} k={k}")
    mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-14, cg_max_it=1000)
    x = torch.from_numpy(x0).cuda()
    mg.smooth(x, torch.from_numpy(b).cuda())
    its, solves = mg.cg_stats()
    assert solves == (n - 1) ** 3
    e = rel_err(x.cpu().numpy(), xref)
    assert e <= 1e-10, (n, k, e, its / max(solves, 1))
    if n == 4:
        announce("patch_smooth f32", f"n={n} k={k}")
        mg32 = StokesMG(n, k, n_levels=1, cg_rtol=1e-6, cg_max_it=300)
        x = torch.from_numpy(x0).float().cuda()
        mg32.smooth(x, torch.from_numpy(b).float().cuda())
        assert rel_err(x.double().cpu().numpy(), xref) <= 1e-4


def test_f32_tight_local_tolerance_stays_finite():
    """A local CG tolerance below FP32 precision (1e-8): the iteration
    stagnates at rounding level and stops when d.Sd is no longer positive,
    instead of dividing by it; the sweep stays finite and close to the FP64
    result."""
    torch = need_gpu()
    n, k = 8, 2
    mg64 = StokesMG(n, k, n_levels=1, cg_rtol=1e-12, cg_max_it=200)
    N = mg64.ndof()
    x0 = uniform_vector(N, seed=5)
    b = uniform_vector(N, seed=6)
    announce("f32 tight local tolerance")
    x64 = torch.from_numpy(x0).cuda()
    mg64.smooth(x64, torch.from_numpy(b).cuda())
    mg32 = StokesMG(n, k, n_levels=1, cg_rtol=1e-8, cg_max_it=200)
    x32 = torch.from_numpy(x0).float().cuda()
    mg32.smooth(x32, torch.from_numpy(b).float().cuda())
    assert torch.isfinite(x32).all()
    assert rel_err(x32.double().cpu().numpy(), x64.cpu().numpy()) <= 1e-4
