"""Writes mixed16_k2_oracle.json: the oracle's solution of the manufactured
sine problem on 16^3 cells, RT_2 / DG Q_2 (435,456 unknowns), used by the
GPU test of the mixed-precision solve at that size.

Calls only the oracle (test infrastructure): FGMRES(30) right-preconditioned
by the oracle's V-cycle (exact pseudo-inverse local solves), iterated to a
relative residual of 1e-12, so the result is the discrete solution to about
that accuracy.  Stored: the residual history, the L2 errors against the
exact solution, the integral mean of the pressure, and the solution at 2000
indices drawn from PCG64(16) plus the first and last index of every block.

Usage (repo root): python tests/golden/make_mixed16_reference.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np

import manufactured as mf
from oracle.mg import Multigrid, fgmres


def main():
    n, k = 16, 2
    t0 = time.time()
    mg = Multigrid(n, k)
    S, K = mg.fine["S"], mg.fine["K"]
    b = S.rhs(mf.sine_f, mf.sine_u)
    x, hist = fgmres(lambda v: K @ v, b, lambda v: mg.vcycle(v), rtol=1e-12)
    x = S.normalize_pressure(x)
    res = float(np.linalg.norm(b - K @ x) / np.linalg.norm(b))
    eu, ep = S.l2_errors(x, mf.sine_u, mf.sine_p)
    rng = np.random.default_rng(16)
    edges = []
    for o in list(S.offsets) + [S.ndof]:
        edges += [o - 1, o]
    idx = np.unique(np.clip(np.concatenate([rng.integers(0, S.ndof, 2000), edges]), 0, S.ndof - 1))
    out = {
        "_source": "tests/golden/make_mixed16_reference.py (oracle only)",
        "problem": "manufactured sine problem (u = curl(sin(pi x) sin(pi y) sin(pi z) (1,1,1)), "
                   "p = cos(pi x) cos(pi y) cos(pi z)), tangential trace imposed weakly",
        "n": n, "k": k, "ndof": int(S.ndof),
        "rtol": 1e-12, "history": [float(h) for h in hist], "rel_residual": res,
        "l2_error_u": float(eu), "l2_error_p": float(ep),
        "pressure_mean": float(S.pressure_mean(x)),
        "max_abs": float(np.abs(x).max()),
        "indices": [int(i) for i in idx],
        "values": [float(v) for v in x[idx]],
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "mixed16_k2_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote mixed16_k2_oracle.json: {len(hist) - 1} steps, residual {res:.2e}, {out['seconds']:.0f} s")


if __name__ == "__main__":
    main()
