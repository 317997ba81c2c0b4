"""The Schur-CG local solver with the in-plane eigenbasis products of the fast
diagonalization on the matrix cores (BF16 operands, FP32 accumulation;
Eqs. inverse2d / fast_inverse, with the mixed precision of Sec. 4.3 carried
into the local solve), in an FP32 cycle.  Against the oracle's sweep with
pseudo-inverse local solves, and inside the mixed-precision solve."""
import numpy as np
import pytest

from gpu_common import need_gpu, announce, rel_err
from oracle.mg import Multigrid
from paper_2410_09497_amd import StokesMG, StokesMGError
from paper_2410_09497_amd.synth import uniform_vector

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,k", [(8, 1), (8, 2), (8, 3), (4, 2)])
def test_fd_bf16_sweep_matches_oracle(n, k):
    """One FP32 sweep with a tight local CG.  A^-1 is applied with two
    BF16-rounded in-plane products (each term with one 2^-9 rounding per
    operand, 2^-8 at first order, FP32 accumulation); the CG solves the Schur
    system of that perturbed A^-1.  Measured 1.8e-3 .. 2.2e-3 relative error
    of the correction; bound 2^-7 (two perturbed products).  The same sweep
    with every product in FP32 stays within 1e-4 (measured 1.1e-6 .. 1.4e-6)."""
    torch = need_gpu()
    mg_o = Multigrid(n, k, n_coarse=n)
    S = mg_o.fine["S"]
    x0 = uniform_vector(S.ndof, seed=90 + k)
    b = uniform_vector(S.ndof, seed=95 + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    dref = mg_o.smooth(0, x0, b) - x0
    mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-6, cg_max_it=200)
    out = {}
    for solver in ("exact", "exact_bf16"):
        announce("fd bf16 sweep", f"n={n} k={k} solver={solver}")
        mg.set_local_solver(solver)
        x = torch.from_numpy(x0).cuda().float()
        mg.smooth(x, torch.from_numpy(b).cuda().float())
        out[solver] = rel_err(x.double().cpu().numpy() - x0, dref)
        print(f"n={n} k={k} {solver}: relative error of the FP32 sweep's correction {out[solver]:.2e}", flush=True)
    mg.set_local_solver("exact")
    assert out["exact"] <= 1e-4
    assert out["exact_bf16"] <= 2.0 ** -7


def test_fd_bf16_solve_converges_like_exact():
    """FP64 FGMRES with an FP32 V-cycle whose local Schur CG uses the BF16
    in-plane products: 1e-8 on 32^3 cells, k = 2, in at most one step more
    than with the FP32 products, and the local CG iterations per patch are
    reported."""
    torch = need_gpu()
    n, k = 32, 2
    mg = StokesMG(n, k, cg_rtol=1e-3, cg_max_it=15)
    b = mg.rhs_manufactured()
    announce("fd bf16 solve", f"n={n} k={k}")
    _, ie = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
    mg.set_local_solver("exact_bf16")
    _, ib = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
    mg.set_local_solver("exact")
    cg = lambda i: i["cg_iterations"] / max(i["local_solves"], 1)
    print(f"FP32 products: {ie['iterations']} steps, {cg(ie):.2f} CG per patch; "
          f"BF16 products: {ib['iterations']} steps, {cg(ib):.2f} CG per patch", flush=True)
    assert ib["converged"] and ib["rel_residual"] <= 1e-8
    assert ib["iterations"] <= ie["iterations"] + 1


def test_fd_bf16_rejects_fp64_and_high_degree():
    torch = need_gpu()
    mg = StokesMG(4, 2, n_levels=1)
    mg.set_local_solver("exact_bf16")
    x = torch.zeros(mg.ndof(), dtype=torch.float64, device="cuda")
    with pytest.raises(StokesMGError):
        mg.smooth(x, x.clone())
    mg.set_local_solver("exact")
    mg4 = StokesMG(4, 4, n_levels=1)
    with pytest.raises(StokesMGError):
        mg4.set_local_solver("exact_bf16")
