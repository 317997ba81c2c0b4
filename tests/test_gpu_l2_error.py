"""stokesmg_l2_error (the library's L2 errors against the manufactured sine
problem, used by the error-versus-time study) against the oracle's
l2_errors of the same vector: the same Gauss rule (k+3 points per
direction), so the two agree to rounding; and the velocity error of the
GPU solution falls like h^(k+1) (O(h^{k+1}), Sec. 3.3)."""
import numpy as np
import pytest

import manufactured as mf
from gpu_common import need_gpu, announce
from oracle.stokes import Stokes
from paper_2410_09497_amd import StokesMG

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,k", [(4, 1), (4, 2), (8, 2), (4, 3)])
def test_l2_error_matches_oracle(n, k):
    torch = need_gpu()
    announce("l2 error", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-12, cg_max_it=300)
    b = mg.rhs_manufactured()
    x, info = mg.solve(b, rtol=1e-10)
    eu, ep = mg.l2_error(x)
    S = Stokes(n, k)
    eu_o, ep_o = S.l2_errors(x.cpu().numpy(), mf.sine_u, mf.sine_p)
    assert abs(eu - eu_o) <= 1e-10 * eu_o and abs(ep - ep_o) <= 1e-10 * ep_o, (eu, eu_o, ep, ep_o)


@pytest.mark.parametrize("k", [1, 2])
def test_velocity_error_order(k):
    torch = need_gpu()
    errs = []
    for n in (8, 16, 32):
        announce("l2 order", f"n={n} k={k}")
        mg = StokesMG(n, k, cg_rtol=1e-10, cg_max_it=300)
        x, info = mg.solve(mg.rhs_manufactured(), rtol=1e-11)
        errs.append(mg.l2_error(x)[0])
    rate = np.log2(errs[-2] / errs[-1])
    print(f"k={k}: velocity errors {errs}, last rate {rate:.2f}", flush=True)
    assert abs(rate - (k + 1)) <= 0.25
