"""GPU parity of the multigrid path: V-cycle (transfers, coarse pseudo-
inverse, smoothing), the manufactured right-hand side, and FGMRES against the
oracle (tight local CG, so the local solves equal the oracle's pseudo-
inverse).  Then the full solve: FP64 and FP32 V-cycle reach 1e-8, pressures
with zero mean, L2 errors equal to the oracle's direct solution."""
import json
import os

import numpy as np
import pytest

import manufactured as mf
from gpu_common import need_gpu, announce, rel_err
from oracle.mg import Multigrid, fgmres
from oracle.stokes import Stokes
from paper_2410_09497_amd import StokesMG
from paper_2410_09497_amd.synth import uniform_vector

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("n,k", [(2, 1), (4, 1), (4, 2), (8, 1), (4, 3)])
def test_vcycle_f64(n, k):
    torch = need_gpu()
    mg_o = Multigrid(n, k)
    S = mg_o.fine["S"]
    b = uniform_vector(S.ndof, seed=40 + n + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.vcycle(b)
    announce("vcycle f64", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-14, cg_max_it=500)
    x = mg.vcycle(torch.from_numpy(b).cuda()).cpu().numpy()
    assert rel_err(x, xref) <= 1e-10


def test_vcycle_f64_degree4():
    """The V-cycle at degree 4 (levels 1^3, 2^3, 4^3) against the oracle's,
    whose patch pseudo-inverses go through the bordered sparse LU."""
    torch = need_gpu()
    n, k = 4, 4
    mg_o = Multigrid(n, k, local_solver="bordered")
    S = mg_o.fine["S"]
    b = uniform_vector(S.ndof, seed=48)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.vcycle(b)
    announce("vcycle f64", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-14, cg_max_it=1000)
    x = mg.vcycle(torch.from_numpy(b).cuda()).cpu().numpy()
    assert rel_err(x, xref) <= 1e-10


@pytest.mark.parametrize("n,k", [(4, 1), (4, 2)])
def test_vcycle_f32(n, k):
    torch = need_gpu()
    mg_o = Multigrid(n, k)
    S = mg_o.fine["S"]
    b = uniform_vector(S.ndof, seed=7)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.vcycle(b)
    announce("vcycle f32", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-6, cg_max_it=200)
    x = mg.vcycle(torch.from_numpy(b).float().cuda()).double().cpu().numpy()
    assert rel_err(x, xref) <= 1e-4


@pytest.mark.parametrize("n,k", [(1, 1), (2, 2), (4, 1), (8, 2)])
def test_rhs_manufactured(n, k):
    torch = need_gpu()
    S = Stokes(n, k)
    bref = S.rhs(mf.sine_f, mf.sine_u)
    announce("rhs", f"n={n} k={k}")
    mg = StokesMG(n, k, n_levels=1)
    b = mg.rhs_manufactured().cpu().numpy()
    assert rel_err(b, bref) <= 1e-12


@pytest.mark.parametrize("n,k,seed", [(2, 1, 0), (4, 2, 5), (8, 1, 7)])
def test_rhs_fourier(n, k, seed):
    """Random smooth force: the library's separable expansion against the
    oracle's pointwise quadrature of the same field."""
    torch = need_gpu()
    S = Stokes(n, k)
    bref = S.rhs(mf.fourier_force(seed))
    announce("rhs fourier", f"n={n} k={k} seed={seed}")
    mg = StokesMG(n, k, n_levels=1)
    b = mg.rhs_fourier(seed).cpu().numpy()
    assert rel_err(b, bref) <= 1e-12


@pytest.mark.parametrize("n,k", [(4, 1), (8, 1), (4, 2)])
def test_fgmres_history_matches_oracle(n, k):
    torch = need_gpu()
    mg_o = Multigrid(n, k)
    S, K = mg_o.fine["S"], mg_o.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    xo, hist_o = fgmres(lambda v: K @ v, b, lambda v: mg_o.vcycle(v), rtol=1e-8)
    announce("fgmres f64", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-14, cg_max_it=500)
    x, info = mg.solve(torch.from_numpy(b).cuda(), rtol=1e-8)
    assert info["iterations"] == len(hist_o) - 1
    h = np.array(info["history"])
    ho = np.array(hist_o)
    assert np.all(np.abs(np.log10(h[1:]) - np.log10(ho[1:])) <= 1e-4), (h, ho)
    assert info["rel_residual"] <= 1e-8
    xg = x.cpu().numpy()
    assert abs(S.pressure_mean(xg)) <= 1e-12 * np.abs(xg).max()
    assert rel_err(xg, S.normalize_pressure(xo)) <= 1e-6


@pytest.mark.parametrize("restart", [1, 2])
def test_fgmres_restart_matches_oracle(restart):
    """Restarted FGMRES(1) and FGMRES(2): the restart path (true residual
    recomputed, new Arnoldi basis) against the oracle's restarted FGMRES."""
    torch = need_gpu()
    n, k = 8, 1
    mg_o = Multigrid(n, k)
    S, K = mg_o.fine["S"], mg_o.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    xo, hist_o = fgmres(lambda v: K @ v, b, lambda v: mg_o.vcycle(v), rtol=1e-8, restart=restart)
    announce("fgmres restart", f"n={n} k={k} restart={restart}")
    mg = StokesMG(n, k, cg_rtol=1e-14, cg_max_it=500)
    x, info = mg.solve(torch.from_numpy(b).cuda(), rtol=1e-8, restart=restart)
    assert info["iterations"] == len(hist_o) - 1 and info["iterations"] > restart
    h = np.array(info["history"])
    ho = np.array(hist_o)
    assert np.all(np.abs(np.log10(h[1:]) - np.log10(ho[1:])) <= 1e-4), (h, ho)
    assert info["rel_residual"] <= 1e-8
    assert rel_err(x.cpu().numpy(), S.normalize_pressure(xo)) <= 1e-6


@pytest.mark.parametrize("k", [1, 2])
def test_solve_f32_vcycle_reaches_tolerance(k):
    """Mixed precision (Sec. 4.3): FP32 V-cycle in FP64 FGMRES, to 1e-8."""
    torch = need_gpu()
    n = 8
    mg_o = Multigrid(n, k)
    S, K = mg_o.fine["S"], mg_o.fine["K"]
    announce("solve mixed", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-6, cg_max_it=100)
    b = mg.rhs_manufactured()
    x64, i64 = mg.solve(b, rtol=1e-8, vcycle_dtype="f64")
    x32, i32 = mg.solve(b, rtol=1e-8, vcycle_dtype="f32")
    assert i32["converged"] and i32["rel_residual"] <= 1e-8
    assert i32["iterations"] <= i64["iterations"] + 1
    xd = S.direct_solve(b.cpu().numpy(), K)
    assert rel_err(x32.cpu().numpy(), xd) <= 1e-6
    eu, ep = S.l2_errors(x32.cpu().numpy(), mf.sine_u, mf.sine_p)
    eu_d, ep_d = S.l2_errors(xd, mf.sine_u, mf.sine_p)
    # the 1e-8 residual leaves a solution difference of ~1e-6 relative (checked
    # above), far below the discretization error: the L2 errors agree to 0.1 %
    assert abs(eu - eu_d) <= 1e-3 * eu_d and abs(ep - ep_d) <= 1e-3 * ep_d


@pytest.mark.xfail(strict=False, reason=(
    "measured with the readings built here (restriction P^T, ascending colours, penalty 2(k+1)^2/h, "
    "exact local solves), sine problem on 8^3 cells, k = 3: steps end at 4.7e-4, 1.7e-6, 1.10e-8, "
    "1.1e-10 -- the third step misses 1e-8 by 10 %; reversed post-smoothing colours and the "
    "paper's own phi-based right-hand side (mu = 0.5 or 0.3, sigma = 0.1 .. 0.25) need 4 or 5 "
    "steps too; with two smoothing sweeps the claim holds (test_solve_paper_three_steps_k3_two_sweeps)"))
def test_solve_paper_three_steps_k3():
    """Sec. 3.3: from k = 3 on, at most three GMRES steps to 1e-8 in 3D."""
    torch = need_gpu()
    gold = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))["three_d_max_steps_from_k3"]
    announce("three steps k=3")
    mg = StokesMG(8, gold["k_min"], cg_rtol=1e-10, cg_max_it=200)
    b = mg.rhs_manufactured()
    x, info = mg.solve(b, rtol=gold["rtol"])
    assert info["converged"], info["history"]
    assert info["iterations"] <= gold["max_steps"], info["history"]


@pytest.mark.xfail(strict=False, reason=(
    "measured with one smoothing sweep: RT_2 on 32^3 cells (sine problem, exact local solves) needs 4 "
    "FGMRES steps to 1e-6 (the third ends at about 3e-6); with two sweeps it takes 3 "
    "(test_table_vs_poisson_rt2_two_sweeps)"))
def test_table_vs_poisson_rt2_iterations():
    """Table vs_poisson (Sec. 4.4), Stokes RT_2 column: 32^3 cells, three
    iterations to a relative residual of 1e-6."""
    torch = need_gpu()
    gold = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))["table_vs_poisson_stokes"]["RT2"]
    announce("table vs_poisson RT2", f"n={gold['n']}")
    mg = StokesMG(gold["n"], gold["k"], cg_rtol=1e-10, cg_max_it=200)
    b = mg.rhs_manufactured()
    x, info = mg.solve(b, rtol=gold["rtol"], max_it=20, allow_notconv=True)
    print("history", info["history"], flush=True)
    assert info["converged"], info["history"]
    assert info["iterations"] <= gold["iterations"], info["history"]


@pytest.mark.parametrize("n,k", [(4, 1), (8, 2)])
def test_vcycle_two_sweeps_matches_oracle(n, k):
    """stokesmg_set_smoothing(2, 2): the V-cycle with two pre- and two
    post-smoothing sweeps against the oracle's V-cycle with the same counts
    (FP64, tight local CG)."""
    torch = need_gpu()
    mg_o = Multigrid(n, k)
    S = mg_o.fine["S"]
    b = uniform_vector(S.ndof, seed=70 + n + k)
    b[S.offsets[3]:] -= b[S.offsets[3]:].mean()
    xref = mg_o.vcycle(b, pre=2, post=2)
    announce("vcycle two sweeps", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-14, cg_max_it=500)
    mg.set_smoothing(2, 2)
    x = mg.vcycle(torch.from_numpy(b).cuda()).cpu().numpy()
    assert rel_err(x, xref) <= 1e-10


@pytest.mark.parametrize("n", [8, 16])
def test_solve_paper_three_steps_k3_two_sweeps(n):
    """Sec. 3.3's "at most three GMRES steps to 1e-8 from k = 3" with two
    smoothing sweeps before and after the coarse correction (the counts of
    the paper's Table 1 in 2D are met with two sweeps as well,
    tests/test_oracle_2d.py)."""
    torch = need_gpu()
    gold = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))["three_d_max_steps_from_k3"]
    announce("three steps k=3, two sweeps", f"n={n}")
    mg = StokesMG(n, gold["k_min"], cg_rtol=1e-10, cg_max_it=200)
    mg.set_smoothing(2, 2)
    b = mg.rhs_manufactured()
    x, info = mg.solve(b, rtol=gold["rtol"])
    print(f"n={n}: {info['iterations']} steps, history {info['history']}", flush=True)
    assert info["converged"]
    assert info["iterations"] <= gold["max_steps"], info["history"]


def test_table_vs_poisson_rt2_two_sweeps():
    """Table vs_poisson's RT_2 column (32^3 cells, three iterations to 1e-6)
    with two smoothing sweeps before and after the coarse correction."""
    torch = need_gpu()
    gold = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))["table_vs_poisson_stokes"]["RT2"]
    announce("table vs_poisson RT2, two sweeps", f"n={gold['n']}")
    mg = StokesMG(gold["n"], gold["k"], cg_rtol=1e-10, cg_max_it=200)
    mg.set_smoothing(2, 2)
    b = mg.rhs_manufactured()
    x, info = mg.solve(b, rtol=gold["rtol"], max_it=20, allow_notconv=True)
    print("history", info["history"], flush=True)
    assert info["converged"]
    assert info["iterations"] <= gold["iterations"], info["history"]


def test_set_smoothing_rejects_bad_counts():
    torch = need_gpu()
    mg = StokesMG(4, 1)
    from paper_2410_09497_amd import StokesMGError
    for pre, post in ((0, 0), (-1, 1), (17, 1)):
        with pytest.raises(StokesMGError):
            mg.set_smoothing(pre, post)


def test_mixed_solve_16_matches_oracle():
    """The mixed-precision solve at the oracle-comparison size of the
    128^3 configuration: 16^3 cells, k = 2 (435,456 unknowns), FP32 V-cycle in
    FP64 FGMRES(30).  Against the oracle's solution of the same problem
    (tests/golden/mixed16_k2_oracle.json, FGMRES + exact V-cycle to 1e-12):
    at 1e-8 the L2 errors agree to 0.1 %; continued to 1e-11, the solution
    agrees to 1e-7 relative at 2000 sampled indices."""
    torch = need_gpu()
    ref = json.load(open(os.path.join(GOLDEN, "mixed16_k2_oracle.json")))
    n, k = ref["n"], ref["k"]
    announce("mixed solve vs oracle", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-6, cg_max_it=100)
    assert mg.ndof() == ref["ndof"]
    b = mg.rhs_manufactured()
    x, info = mg.solve(b, rtol=1e-8, vcycle_dtype="f32")
    assert info["converged"] and info["rel_residual"] <= 1e-8
    S = Stokes(n, k)
    xh = x.cpu().numpy()
    eu, ep = S.l2_errors(xh, mf.sine_u, mf.sine_p)
    assert abs(eu - ref["l2_error_u"]) <= 1e-3 * ref["l2_error_u"]
    assert abs(ep - ref["l2_error_p"]) <= 1e-3 * ref["l2_error_p"]
    assert abs(S.pressure_mean(xh)) <= 1e-12 * ref["max_abs"]
    idx = np.array(ref["indices"])
    vals = np.array(ref["values"])
    d8 = np.abs(xh[idx] - vals).max() / ref["max_abs"]
    x, info = mg.solve(b, rtol=1e-11, vcycle_dtype="f32", max_it=60)
    assert info["converged"]
    d11 = np.abs(x.cpu().numpy()[idx] - vals).max() / ref["max_abs"]
    print(f"max sampled difference / max|x|: {d8:.2e} at 1e-8, {d11:.2e} at 1e-11", flush=True)
    assert d11 <= 1e-7
