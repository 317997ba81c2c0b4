"""The Direct local solver (Sec. 3.3) on the matrix cores: every patch of a
colour in one launch that gathers the patch residuals, multiplies them by
the normalized pseudo-inverse of their patch type (interior, face, edge,
corner; the single patch of n = 2) and scatters the corrections.
Against the oracle's smoother with pseudo-inverse local solves on every
patch, and inside the mixed-precision solve."""
import numpy as np
import pytest

from gpu_common import need_gpu, announce, rel_err
from oracle.mg import Multigrid
from paper_2410_09497_amd import StokesMG
from paper_2410_09497_amd.synth import uniform_vector

pytestmark = pytest.mark.gpu


def _direct_mg(n, k, levels=None, cg_rtol=1e-12, cg_max_it=300):
    mg = StokesMG(n, k, n_levels=levels, cg_rtol=cg_rtol, cg_max_it=cg_max_it)
    mg.mlp_setup(1024)
    mg.direct_setup()
    return mg


CASES = [(8, 1), (8, 2), (8, 3),
         # n = 4: every patch touches the boundary (all 27 types, vertices 1..3)
         (4, 2),
         # n = 2: the single patch, boundary on all six outer faces
         (2, 1), (2, 2)]


@pytest.mark.parametrize("n,k", CASES)
def test_direct_sweep_matches_oracle(n, k):
    """One sweep.  The GEMM rounds the normalized residuals and the matrix to
    its operand precision and accumulates in FP32; every patch of the sweep
    goes through it.  Each product term carries at most one rounding of
    each operand, 2 u relative at first order, and the errors of the d terms
    have independent signs.  FP32 operands (u = 2^-24) leave 2e-7 .. 4e-7
    relative error in the sweep's correction (bound 1e-6, FP32 accumulation
    and the eight colours included); BF16 operands (u = 2^-9) 1.3e-3 ..
    2.8e-3 (bound: the first-order worst case of one term, 2^-8 = 3.9e-3)."""
    torch = need_gpu()
    mg_o = Multigrid(n, k, n_coarse=n)
    S = mg_o.fine["S"]
    x0 = uniform_vector(S.ndof, seed=50 + k)
    b = uniform_vector(S.ndof, seed=60 + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.smooth(0, x0, b)
    dref = xref - x0
    mg = _direct_mg(n, k, levels=1)
    for mode, tol in (("f32", 1e-6), ("bf16", 2.0 ** -8)):
        announce("direct sweep", f"n={n} k={k} mode={mode}")
        mg.set_local_solver("direct", mode)
        x = torch.from_numpy(x0).cuda()
        mg.smooth(x, torch.from_numpy(b).cuda())
        e = rel_err(x.cpu().numpy() - x0, dref)
        print(f"n={n} k={k} {mode}: relative error of the sweep's correction {e:.2e}", flush=True)
        assert e <= tol, (k, mode, e)
    mg.set_local_solver("exact")


@pytest.mark.parametrize("k", [1, 2, 3])
def test_direct_sweep_full_size_matches_exact_sweep(k):
    """64^3 cells, where the kernel runs 128 x 128 tiles (the 8^3 cases run
    64 x 64): one Direct sweep against one sweep of the exact local solver
    (FP64 Schur CG to 1e-12, itself checked against the oracle at small
    sizes), same seeded inputs, same bounds as above."""
    torch = need_gpu()
    n = 64
    mg = _direct_mg(n, k, levels=1)
    N = mg.ndof()
    x0 = torch.from_numpy(uniform_vector(N, seed=70 + k)).cuda()
    b = torch.from_numpy(uniform_vector(N, seed=80 + k)).cuda()
    announce("direct sweep vs exact", f"n={n} k={k}")
    mg.set_local_solver("exact")
    xe = x0.clone()
    mg.smooth(xe, b)
    de = (xe - x0).cpu().numpy()
    for mode, tol in (("f32", 1e-6), ("bf16", 2.0 ** -8)):
        mg.set_local_solver("direct", mode)
        x = x0.clone()
        mg.smooth(x, b)
        e = rel_err((x - x0).cpu().numpy(), de)
        print(f"n={n} k={k} {mode}: relative difference to the exact sweep {e:.2e}", flush=True)
        assert e <= tol, (k, mode, e)
    mg.set_local_solver("exact")


def test_direct_solve_converges_like_exact():
    """FP64 FGMRES with an FP32 V-cycle whose local solves are all the Direct
    GEMM (BF16 or FP32 operands): reaches 1e-8 on 32^3 cells, k = 2, in at
    most one step more than the exact local solver."""
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
