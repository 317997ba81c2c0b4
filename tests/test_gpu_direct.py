"""The Direct local solver (Sec. 3.3) on the matrix cores: interior patches
by one GEMM per batch with the normalized patch pseudo-inverse, boundary
patches by the Schur CG.  Against the oracle's smoother with pseudo-inverse
local solves on every patch, and inside the mixed-precision solve."""
import numpy as np
import pytest

from gpu_common import need_gpu, announce, rel_err
from oracle.mg import Multigrid
from paper_2410_09497_amd import StokesMG
from paper_2410_09497_amd.synth import uniform_vector

pytestmark = pytest.mark.gpu


def _direct_mg(n, k, levels=None, cg_rtol=1e-12, cg_max_it=300):
    mg = StokesMG(n, k, n_levels=levels, cg_rtol=cg_rtol, cg_max_it=cg_max_it)
    mg.mlp_setup(4096)
    mg.direct_setup()
    return mg


@pytest.mark.parametrize("k", [1, 2, 3])
def test_direct_sweep_matches_oracle(k):
    """One sweep at 8^3 cells (interior patches 2 <= v <= 6).  The GEMM
    rounds the normalized residuals and the matrix to its operand precision
    and accumulates in FP32.  FP32 operands (rounding 2^-24) leave about 5e-8
    relative error in the sweep's correction (bound 1e-6); BF16 operands
    (rounding 2^-9 = 2e-3 per operand, errors of independent sign over
    d >= 208 terms) about 2e-4 (bound: one BF16 rounding unit, 2e-3)."""
    torch = need_gpu()
    n = 8
    mg_o = Multigrid(n, k, n_coarse=n)
    S = mg_o.fine["S"]
    x0 = uniform_vector(S.ndof, seed=50 + k)
    b = uniform_vector(S.ndof, seed=60 + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.smooth(0, x0, b)
    dref = xref - x0
    mg = _direct_mg(n, k, levels=1)
    for mode, tol in (("f32", 1e-6), ("bf16", 2e-3)):
        announce("direct sweep", f"n={n} k={k} mode={mode}")
        mg.set_local_solver("direct", mode)
        x = torch.from_numpy(x0).cuda()
        mg.smooth(x, torch.from_numpy(b).cuda())
        e = rel_err(x.cpu().numpy() - x0, dref)
        print(f"k={k} {mode}: relative error of the sweep's correction {e:.2e}", flush=True)
        assert e <= tol, (k, mode, e)
    mg.set_local_solver("exact")


def test_direct_solve_converges_like_exact():
    """FP64 FGMRES with an FP32 V-cycle whose interior local solves are the
    BF16 Direct GEMM: reaches 1e-8 on 32^3 cells, k = 2, in at most one step
    more than the exact local solver."""
    torch = need_gpu()
    n, k = 32, 2
    mg = StokesMG(n, k, cg_rtol=1e-3, cg_max_it=15)
    mg.mlp_setup(65536)
    mg.direct_setup()
    b = mg.rhs_manufactured()
    announce("direct solve", f"n={n} k={k}")
    _, ie = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
    out = {}
    for mode in ("bf16", "f32"):
        mg.set_local_solver("direct", mode)
        _, info = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
        out[mode] = info
        print(f"{mode}: {info['iterations']} steps vs exact {ie['iterations']}", flush=True)
        assert info["converged"] and info["rel_residual"] <= 1e-8
        assert info["iterations"] <= ie["iterations"] + 1
    mg.set_local_solver("exact")


def test_direct_needs_setup():
    torch = need_gpu()
    mg = StokesMG(8, 2)
    from paper_2410_09497_amd import StokesMGError
    mg.mlp_setup(1024)
    with pytest.raises(StokesMGError):
        mg.set_local_solver("direct", "bf16")
