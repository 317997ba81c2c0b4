"""Solve the manufactured Stokes problem on the unit cube and print the
outcome, one JSON line per solve:

    python -m paper_2410_09497_amd.run_solve --n 64 --k 2 --vcycle f64
    python paper_2410_09497_amd/run_solve.py --n 128 --k 2 --vcycle f32 --local exact direct

u = curl(sin(pi x) sin(pi y) sin(pi z) (1,1,1)), p = cos(pi x) cos(pi y) cos(pi z);
FGMRES(restart) preconditioned by the V-cycle down to 1^3 cells.  --local
lists the local solvers to run one after the other: exact (Schur CG
everywhere), exact_bf16 (the Schur CG with its in-plane eigenbasis products
on the matrix cores, FP32 cycle) and direct (every patch by the Direct solver
on the matrix cores, BF16 operands unless --operands f32).  L2 errors of every solution
are printed too."""
import argparse
import json
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--vcycle", choices=["f64", "f32"], default="f64")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=8)
    ap.add_argument("--cg-rtol", type=float, default=1e-3)
    ap.add_argument("--cg-max-it", type=int, default=15)
    ap.add_argument("--local", nargs="+", choices=["exact", "exact_bf16", "direct"], default=["exact"])
    ap.add_argument("--operands", choices=["bf16", "f32"], default="bf16")
    args = ap.parse_args()
    from paper_2410_09497_amd import StokesMG
    mg = StokesMG(args.n, args.k, cg_rtol=args.cg_rtol, cg_max_it=args.cg_max_it)
    if "direct" in args.local:
        mg.mlp_setup(131072)
        mg.direct_setup()
    b = mg.rhs_manufactured()
    for local in args.local:
        mg.set_local_solver(local, args.operands)
        x, info = mg.solve(b, rtol=args.rtol, restart=args.restart, vcycle_dtype=args.vcycle)
        eu, ep = mg.l2_error(x)
        print(json.dumps({"n": args.n, "k": args.k, "vcycle": args.vcycle, "local_solver": local,
                          "operands": args.operands if local == "direct" else ("bf16" if local == "exact_bf16" else None),
                          "unknowns": mg.ndof(),
                          "iterations": info["iterations"], "seconds": info["seconds"],
                          "rel_residual": info["rel_residual"], "nu": info["nu"], "l2_error_u": eu,
                          "l2_error_p": ep}), flush=True)
    mg.set_local_solver("exact")


if __name__ == "__main__":
    main()
