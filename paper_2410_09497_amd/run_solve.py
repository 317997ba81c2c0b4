"""Solve the manufactured Stokes problem on the unit cube and print the
outcome: python -m paper_2410_09497_amd.run_solve --n 64 --k 2 --vcycle f64

u = curl(sin(pi x) sin(pi y) sin(pi z) (1,1,1)), p = cos(pi x) cos(pi y) cos(pi z);
FGMRES(restart) preconditioned by the V-cycle down to 1^3 cells."""
import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--vcycle", choices=["f64", "f32"], default="f64")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--cg-rtol", type=float, default=1e-3)
    ap.add_argument("--cg-max-it", type=int, default=15)
    args = ap.parse_args()
    from . import StokesMG
    mg = StokesMG(args.n, args.k, cg_rtol=args.cg_rtol, cg_max_it=args.cg_max_it)
    b = mg.rhs_manufactured()
    _, info = mg.solve(b, rtol=args.rtol, restart=args.restart, vcycle_dtype=args.vcycle)
    print(json.dumps({"n": args.n, "k": args.k, "vcycle": args.vcycle, "unknowns": mg.ndof(),
                      "iterations": info["iterations"], "seconds": info["seconds"],
                      "rel_residual": info["rel_residual"], "nu": info["nu"]}), flush=True)


if __name__ == "__main__":
    main()
