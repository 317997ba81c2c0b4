"""Benchmark of the hot path on one MI355X.

Default workload: the plain method at scale, 64^3 cells, RT_2 / DG Q_2
(28,200,960 unknowns), input x ~ U[-1, 1] (PCG64 seed k), FP64.  One step is
one pass of the built hot path over that input: the fused operator
application y = K x (stokes_apply).  `value` is unknowns per second of the
timed steps; `roofline` relates the operator kernel's algorithmic HBM bytes
(read x once, write y once: 16 B per unknown in FP64) to its measured launch
time and to the MI355X HBM peak; `cpu_baseline` times the CPU oracle's
operator on a bounded sample of the same problem family on this host.

Inputs rotate over enough (x, y) pairs that the working set exceeds the
256 MB Infinity Cache, so the figure is an HBM figure.

Second part of the metric, `solve` (k = 2) and `solve_k3` (k = 3): time to
a relative residual of 1e-8 of FGMRES(8) preconditioned by the V-cycle on
128^3 cells (226 M / 536 M unknowns, 8 levels): all-FP64 multigrid, the FP32
V-cycle, the FP32 V-cycle with the Direct local solver on the matrix cores,
and -- on random smooth right-hand sides from an unseen seed -- the learned
local solver with its exact-solver fallback and the network's pressure as
the start of the exact local CG (network trained first on pairs captured
from exact V-cycles on 32^3 cells).

Third part, `c1`: the operator and the smoother for every degree k = 1..5 in
FP64 and FP32 at 64^3 cells (K applications and a few sweeps per cell).
Fourth part, `error_vs_time`: L2 errors against time to solution for
k = 1..4 on 16^3 .. 128^3 cells.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--k 2] [--n 64]
                       [--dtype f64|f32] [--no-cpu-baseline] [--no-solve]
                       [--solve-n 128] [--no-c1] [--c1-sweeps 3] [--no-k3] [--no-f4]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Stokes apply DoF/s (%HBM roofline); time to 1e-8 res, FP64 MG vs FP32/learned MG"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2410_09497_amd/csrc/apply_kernel.hpp", "paper_2410_09497_amd/csrc/apply3_kernel.hpp",
                  "paper_2410_09497_amd/csrc/apply_launch.hpp",
                  "paper_2410_09497_amd/csrc/apply_common.cpp", "paper_2410_09497_amd/csrc/stencil_tables.hpp",
                  "paper_2410_09497_amd/csrc/apply_k{k}.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_traffic.json")


def kernel_source_hash(k):
    """Hash of the sources that define the operator kernel of degree k."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f.format(k=k)), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(k, n, dtype, ndof):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel source; else None."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    key = f"k{k}_n{n}_{dtype}"
    ent = rec.get("cases", {}).get(key)
    if not ent or ent.get("kernel_source_hash") != kernel_source_hash(k):
        return None
    return ent.get("hbm_bytes_per_launch")


def cpu_baseline(k):
    """The oracle's operator (element matrices, NumPy FP64) on 32^3 cells at the
    same degree: a bounded sample (1/8 of the 64^3 mesh).  `cores` is the
    number of cores the oracle kept busy: process CPU time over wall time of
    the timed repetitions (NumPy's BLAS runs the element products on several
    threads; the scatter-add runs on one)."""
    import numpy as np
    from oracle.stokes import Stokes
    from paper_2410_09497_amd.synth import uniform_vector
    n = 32
    S = Stokes(n, k)
    x = uniform_vector(S.ndof, seed=k)
    S.local_matrices()
    S.apply(x)
    reps = 0
    c0 = os.times()
    t0 = time.perf_counter()
    while True:
        S.apply(x)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 3:
            break
    c1 = os.times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    cores = cpu / el
    return {"value": S.ndof * reps / el, "unit": "DoF/s", "cores": round(cores, 1), "kind": "oracle",
            "sample": f"oracle stokes apply (local element matrices, NumPy FP64) on {n}^3 cells, k={k} "
                      f"({S.ndof} unknowns), {reps} repetitions, {el:.1f} s wall, {cpu:.1f} s CPU; host has "
                      f"{len(os.sched_getaffinity(0))} usable cores"}


def c1_section(dev, n, steps, sweeps, log):
    """Every degree and precision of the plain method at scale: the operator
    (steps applications, HIP events on the launch stream, rotating pairs over
    512 MB) and the smoother (sweeps of patch_smooth from x = 0 on a random
    right-hand side, local CG rtol 1e-3 / at most 15 iterations)."""
    import torch
    from paper_2410_09497_amd import StokesMG
    from paper_2410_09497_amd.synth import uniform_vector
    out = {"workload": f"{n}^3 cells, RT_k/DG Q_k, k = 1..5, FP64 and FP32; x ~ U[-1,1] PCG64 seed k; "
                       f"{steps} stokes_apply calls and {sweeps} patch_smooth sweeps per cell of the table"}
    stream = torch.cuda.current_stream(dev)
    for k in range(1, 6):
        mg = StokesMG(n, k, n_levels=1, cg_rtol=1e-3, cg_max_it=15, device=dev)
        ndof = mg.ndof()
        x64 = torch.from_numpy(uniform_vector(ndof, seed=k)).to(dev)
        for dt, es in (("f64", 8), ("f32", 4)):
            x0 = x64 if dt == "f64" else x64.float()
            npairs = max(1, -(-512 * 2 ** 20 // (2 * ndof * es)))
            xs = [x0.clone() for _ in range(npairs)]
            ys = [torch.empty_like(x0) for _ in range(npairs)]
            for i in range(3):
                mg.apply(xs[i % npairs], ys[i % npairs])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(steps):
                mg.apply(xs[i % npairs], ys[i % npairs])
            e1.record(stream)
            torch.cuda.synchronize()
            t_apply = e0.elapsed_time(e1) * 1e-3 / steps
            del xs, ys
            b = x0.clone()
            xsm = torch.zeros_like(x0)
            mg.smooth(xsm, b, sweeps=1)
            mg.cg_stats(reset=True)
            xsm.zero_()
            e0.record(stream)
            mg.smooth(xsm, b, sweeps=sweeps)
            e1.record(stream)
            torch.cuda.synchronize()
            t_sweep = e0.elapsed_time(e1) * 1e-3 / sweeps
            its, solves = mg.cg_stats(reset=True)
            cell = {"unknowns": ndof, "apply_ms": t_apply * 1e3, "apply_GDoF_s": ndof / t_apply / 1e9,
                    "apply_hbm_frac": 2 * es * ndof / t_apply / 1e9 / HBM_PEAK_GBS,
                    "sweep_ms": t_sweep * 1e3, "sweep_GDoF_s": ndof / t_sweep / 1e9,
                    "sweep_avg_local_cg": its / max(solves, 1)}
            if k <= 3 and dt == "f32":
                # the same sweeps with the Direct solver on the interior patches (BF16 operands on MFMA)
                mg.mlp_setup(131072)
                mg.direct_setup()
                mg.set_local_solver("direct", "bf16")
                xsm.zero_()
                mg.smooth(xsm, b, sweeps=1)
                xsm.zero_()
                e0.record(stream)
                mg.smooth(xsm, b, sweeps=sweeps)
                e1.record(stream)
                torch.cuda.synchronize()
                mg.set_local_solver("exact")
                cell["sweep_direct_bf16_ms"] = e0.elapsed_time(e1) / sweeps
            out[f"k{k}_{dt}"] = cell
            log(f"[bench] C1 k={k} {dt}: apply {t_apply * 1e3:.3f} ms, sweep {t_sweep * 1e3:.1f} ms"
                + (f", direct sweep {cell['sweep_direct_bf16_ms']:.1f} ms" if "sweep_direct_bf16_ms" in cell else ""))
        del mg, x64
        torch.cuda.empty_cache()
    return out


def _run(mg, b, log, name, solver="exact", mode="bf16", vcycle="f32", rho_ref=0.0, sweeps=1):
    mg.set_local_solver(solver, mode)
    mg.set_smoothing(sweeps, sweeps)
    if solver == "mlp":
        mg.set_fallback(rho_ref)
    x, info = mg.solve(b, rtol=1e-8, max_it=30, vcycle_dtype=vcycle, restart=8, allow_notconv=True)
    mg.set_local_solver("exact")
    mg.set_smoothing(1, 1)
    out = {"seconds": info["seconds"], "iterations": info["iterations"], "rel_residual": info["rel_residual"],
           "converged": info["converged"], "nu": info["nu"], "history": info["history"],
           "avg_local_cg": info["cg_iterations"] / max(info["local_solves"], 1),
           "local_solver": solver, "vcycle": vcycle, "sweeps": sweeps,
           "operands": "bf16" if solver == "exact_bf16" else (mode if solver != "exact" else None)}
    if solver == "mlp":
        fb = info["fallback_iteration"]
        out.update(fallback_iteration=fb, rho_ref=rho_ref, fallback_bound=max(2 * rho_ref, 1e-3),
                   learned_steps_used=info["iterations"] if fb < 0 else fb)
    log(f"[bench] {name}: {info['seconds']:.3f} s, {info['iterations']} steps, "
        f"avg local CG {out['avg_local_cg']:.2f}")
    return out


def train_network(dev, k, pairs, epochs, log):
    """Pairs (normalized patch residual, exact correction) from exact FP64
    V-cycles on 32^3 cells with random smooth right-hand sides (seeds 0, 1,
    ...), then Adam on the BF16 MFMA kernels."""
    import torch
    from paper_2410_09497_amd import StokesMG
    nt = 32
    tr = StokesMG(nt, k, cg_rtol=1e-10, cg_max_it=200, device=dev)
    tr.mlp_setup(65536)
    tr.mlp_init(seed=0)
    d, _ = tr.mlp_dims()
    X = torch.empty(pairs, d, dtype=torch.float32, device=dev)
    T = torch.empty_like(X)
    cnt, s = 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while cnt < pairs:
        cnt, _ = tr.mlp_collect_pairs(tr.rhs_fourier(seed=s), X, T, n=cnt)
        s += 1
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    batch = 4096
    t0 = time.perf_counter()
    hist = tr.mlp_train(X, T, n=cnt, epochs=epochs, batch=batch, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    d_h = 256
    flop_per_sample = 3 * 2 * (d * d_h + d_h * d_h + d_h * d)
    state, step = tr.mlp_get_state()
    del tr, X, T
    torch.cuda.empty_cache()
    log(f"[bench] training k={k}: {cnt} pairs, {t_train:.2f} s for {epochs} epochs")
    info = {"pairs": cnt, "v_cycles": s, "collect_seconds": t_collect, "epochs": epochs, "batch": batch,
            "train_seconds": t_train, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
            "samples_per_s": epochs * cnt / t_train, "tflops": epochs * cnt * flop_per_sample / t_train / 1e12,
            "mfma_peak_tflops_bf16": 2500.0,
            "workload": f"pairs from exact FP64 V-cycles on {nt}^3 cells, RT_{k}, random smooth right-hand sides "
                        f"(8 Fourier modes per component, wavenumbers 1..8, seeds 0..{s - 1}); MLP {d}-256-256-{d}, "
                        "GELU, BF16 operands, FP32 accumulation, Adam"}
    return state, step, info


def solve_section(dev, k, n_solve, log):
    """Time to 1e-8 (wall time of solve()) of FGMRES(8) with the V-cycle on
    n_solve^3 cells.  The manufactured sine problem: all-FP64 multigrid, the
    FP32 V-cycle, the FP32 V-cycle whose local solves are the Direct solver on
    the matrix cores (BF16 and FP32 operands), and the FP32 V-cycle whose
    Schur CG takes its in-plane eigenbasis products on the matrix cores (BF16
    operands).  Random smooth
    right-hand sides from an unseen seed: the same, plus the learned local
    solver (the network in place of the interior local solves, with the
    exact-solver fallback) and the network's pressure as the start of the
    exact Schur CG."""
    import torch
    from paper_2410_09497_amd import StokesMG

    mg = StokesMG(n_solve, k, cg_rtol=1e-3, cg_max_it=15, device=dev)
    mg.mlp_setup(131072)
    t0 = time.perf_counter()
    mg.direct_setup()
    t_direct = time.perf_counter() - t0
    out = {"workload": f"FGMRES(8) + V(1,1) to 1e-8 on {n_solve}^3 cells, RT_{k}/DG Q_{k}, levels down to 1^3; "
                       "local Schur CG rtol 1e-3, at most 15 iterations",
           "unknowns": mg.ndof(), "direct_setup_seconds": t_direct}
    b = mg.rhs_manufactured()
    sine = {"problem": "manufactured sine problem"}
    sine["fp64_mg"] = _run(mg, b, log, "sine fp64_mg", vcycle="f64")
    sine["fp32_mg"] = _run(mg, b, log, "sine fp32_mg")
    sine["fp32_direct_bf16"] = _run(mg, b, log, "sine fp32_direct_bf16", "direct", "bf16")
    sine["fp32_direct_f32"] = _run(mg, b, log, "sine fp32_direct_f32", "direct", "f32")
    sine["fp32_fd_bf16"] = _run(mg, b, log, "sine fp32_fd_bf16", "exact_bf16")
    # two smoothing sweeps before and after the coarse correction: the sweep count with which the paper's printed
    # iteration counts are met
    sine["fp32_mg_two_sweeps"] = _run(mg, b, log, "sine fp32_mg_two_sweeps", sweeps=2)
    sine["fp32_direct_bf16_two_sweeps"] = _run(mg, b, log, "sine fp32_direct_bf16_two_sweeps", "direct", "bf16",
                                               sweeps=2)
    for v in ("fp32_mg", "fp32_direct_bf16", "fp32_direct_f32", "fp32_fd_bf16", "fp32_mg_two_sweeps",
              "fp32_direct_bf16_two_sweeps"):
        sine[v + "_speedup_vs_fp64"] = sine["fp64_mg"]["seconds"] / sine[v]["seconds"]
    out["sine"] = sine
    h = sine["fp32_mg"]["history"]
    rho_ref = h[-1] ** (1.0 / max(sine["fp32_mg"]["iterations"], 1))

    state, step, tinfo = train_network(dev, k, 1_000_000 if k == 2 else 400_000, 20 if k == 2 else 10, log)
    out["training"] = tinfo
    mg.mlp_set_state(state, step)
    seed = 1_000_000 + 7
    bf = mg.rhs_fourier(seed=seed)
    four = {"problem": f"random smooth right-hand side, unseen seed {seed}"}
    four["fp64_mg"] = _run(mg, bf, log, "fourier fp64_mg", vcycle="f64")
    four["fp32_mg"] = _run(mg, bf, log, "fourier fp32_mg")
    four["fp32_direct_bf16"] = _run(mg, bf, log, "fourier fp32_direct_bf16", "direct", "bf16")
    four["fp32_mlp"] = _run(mg, bf, log, "fourier fp32_mlp", "mlp", "bf16", rho_ref=rho_ref)
    four["fp32_mlp_warm"] = _run(mg, bf, log, "fourier fp32_mlp_warm", "mlp_warm", "bf16")
    for v in ("fp32_mg", "fp32_direct_bf16", "fp32_mlp", "fp32_mlp_warm"):
        four[v + "_speedup_vs_fp64"] = four["fp64_mg"]["seconds"] / four[v]["seconds"]
    fb = four["fp32_mlp"]["fallback_iteration"]
    if fb >= 0:
        four["learned_note"] = (f"the network in place of the local solve: the contraction monitor handed the solve "
                                f"to the exact local solver after {fb} learned step(s)")
    four["warm_note"] = (f"the network's pressure as the start of the exact Schur CG: "
                         f"{four['fp32_mlp_warm']['avg_local_cg']:.2f} local CG iterations per patch against "
                         f"{four['fp32_mg']['avg_local_cg']:.2f} without it, same stopping test")
    out["fourier"] = four
    del mg
    torch.cuda.empty_cache()
    return out


def error_vs_time_section(dev, log):
    """Error against time to solution (the study of Sec. 3.3's 3D figure of
    error over solve time): the manufactured sine problem to 1e-8 with the
    FP32 V-cycle in FP64 FGMRES(8) (interior local solves by the Direct solver
    on the matrix cores for k <= 3, the Schur CG at k = 4), for k = 1..4 on
    16^3 .. 128^3 cells; L2 errors of velocity and pressure by the library's
    quadrature (stokesmg_l2_error)."""
    import torch
    from paper_2410_09497_amd import StokesMG
    out = {"workload": "sine problem to 1e-8, FP32 V-cycle in FP64 FGMRES(8); Direct BF16 interior solves for "
                       "k <= 3; local Schur CG rtol 1e-3 (<= 15 iterations) elsewhere", "runs": []}
    for k in (1, 2, 3, 4):
        for n in (16, 32, 64, 128):
            if (k == 4 and n > 64) or (k == 3 and n > 128):
                continue
            mg = StokesMG(n, k, cg_rtol=1e-3, cg_max_it=15, device=dev)
            solver = "exact"
            if k <= 3:
                mg.mlp_setup(131072)
                mg.direct_setup()
                solver = "direct"
            mg.set_local_solver(solver, "bf16")
            b = mg.rhs_manufactured()
            x, info = mg.solve(b, rtol=1e-8, max_it=30, vcycle_dtype="f32", restart=8)
            eu, ep = mg.l2_error(x)
            out["runs"].append({"k": k, "n": n, "unknowns": mg.ndof(), "seconds": info["seconds"],
                                "iterations": info["iterations"], "l2_error_u": eu, "l2_error_p": ep,
                                "local_solver": solver})
            log(f"[bench] error-vs-time k={k} n={n}: {info['seconds']:.3f} s, {info['iterations']} steps, "
                f"|u-u_h| {eu:.3e}, |p-p_h| {ep:.3e}")
            del mg, x, b
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solve-n", type=int, default=128)
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--c1-sweeps", type=int, default=3)
    ap.add_argument("--no-k3", action="store_true", help="skip the degree-3 solves (C4 at k = 3)")
    ap.add_argument("--no-f4", action="store_true", help="skip the error-versus-time study")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the method's hot path here is single-GPU "
              "(multi-GPU sharding is a design note, not a built path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_09497_amd import StokesMG
    from paper_2410_09497_amd.synth import uniform_vector

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    k, n = args.k, args.n
    tdtype = torch.float64 if args.dtype == "f64" else torch.float32
    es = 8 if args.dtype == "f64" else 4
    mg = StokesMG(n, k, n_levels=1, device=dev)
    ndof = mg.ndof()
    x0 = torch.from_numpy(uniform_vector(ndof, seed=k)).to(dev, tdtype)
    # enough (x, y) pairs that the rotating working set exceeds 2x the Infinity Cache
    pair_bytes = 2 * ndof * es
    npairs = max(1, -(-512 * 2 ** 20 // pair_bytes))
    xs = [x0.clone() for _ in range(npairs)]
    ys = [torch.empty_like(x0) for _ in range(npairs)]

    stream = torch.cuda.current_stream(dev)
    for i in range(args.warmup):
        mg.apply(xs[i % npairs], ys[i % npairs])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.steps):
        mg.apply(xs[i % npairs], ys[i % npairs])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    # every step is exactly one launch of the operator kernel
    launch_s = ms_step * 1e-3
    alg_bytes = 2.0 * es * ndof
    achieved = alg_bytes / launch_s / 1e9

    # plain device-to-device copy of the same byte count, for context
    cbuf_a = torch.empty(ndof, dtype=tdtype, device=dev)
    cbuf_b = torch.empty_like(cbuf_a)
    for _ in range(3):
        cbuf_b.copy_(cbuf_a)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(20):
        cbuf_b.copy_(cbuf_a)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * es * ndof * 20 / (c0.elapsed_time(c1) * 1e-3) / 1e9

    traffic = measured_traffic(k, n, args.dtype, ndof)
    out = {
        "metric": METRIC,
        "value": ndof / launch_s,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"stokes_apply on {n}^3 cells, RT_{k}/DG Q_{k} ({ndof} unknowns), "
                               f"x ~ U[-1,1] PCG64 seed {k}, {npairs} rotating (x, y) pairs",
                   "n_cells": n, "k": k, "unknowns": ndof, "levels": 1},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "stokes_apply (the fused operator kernel dispatched for this degree and dtype)",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "copy_GBps_same_bytes": copy_gbs,
        "context": "paper (A100, FP64): > 1 GDoF/s operator evaluation; 0.535 ns/DoF = 1.87 GDoF/s "
                   "for RT_2 on 32^3 (Table vs_poisson)",
    }
    del xs, ys, cbuf_a, cbuf_b, mg
    torch.cuda.empty_cache()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if not args.no_c1:
        out["c1"] = c1_section(dev, args.n, args.steps, args.c1_sweeps, log)
    if not args.no_solve:
        out["solve"] = solve_section(dev, k, args.solve_n, log)
        if not args.no_k3 and k != 3:
            out["solve_k3"] = solve_section(dev, 3, args.solve_n, log)
    if not args.no_f4:
        out["error_vs_time"] = error_vs_time_section(dev, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(k)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
