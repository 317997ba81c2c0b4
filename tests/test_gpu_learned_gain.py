"""What the trained network gains (the learned part, not in the paper).

The network is trained on the GPU (hand-written forward/backward/Adam
kernels; 10^6 pairs, 20 epochs, as in the benchmark) on pairs captured from
exact V-cycles on 32^3 cells, k = 2, with random smooth right-hand sides
(seeds 0, 1, ...), then used on a right-hand side from an unseen seed:
* as the start of the exact Schur CG on interior patches (the exact solver
  keeps its stopping test, so it judges): the outer FGMRES steps and the
  final residual stay those of the method without the network, and the
  local CG needs fewer iterations per patch -- the gain;
* in place of the interior local solves, with the contraction monitor: the
  solve still reaches 1e-8 (the exact solver takes over when the learned
  steps do not contract enough).
The wall-clock effect at 128^3 cells is reported by the benchmark."""
import pytest

from gpu_common import need_gpu, announce

pytestmark = pytest.mark.gpu


def test_trained_network_saves_local_cg_iterations():
    torch = need_gpu()
    from paper_2410_09497_amd import StokesMG
    n, k = 32, 2
    announce("learned gain: training", f"n={n} k={k}")
    tr = StokesMG(n, k, cg_rtol=1e-10, cg_max_it=200)
    tr.mlp_setup(65536)
    tr.mlp_init(seed=0)
    d, _ = tr.mlp_dims()
    cap = 1_000_000
    X = torch.empty(cap, d, dtype=torch.float32, device="cuda")
    T = torch.empty_like(X)
    cnt, s = 0, 0
    while cnt < cap:
        cnt, _ = tr.mlp_collect_pairs(tr.rhs_fourier(seed=s), X, T, n=cnt)
        s += 1
    hist = tr.mlp_train(X, T, n=cnt, epochs=20, batch=4096, lr=1e-3, seed=1)
    assert hist[-1] < 0.5 * hist[0]
    state, step = tr.mlp_get_state()
    del tr, X, T
    torch.cuda.empty_cache()

    announce("learned gain: solves", f"n={n} k={k}")
    mg = StokesMG(n, k, cg_rtol=1e-3, cg_max_it=15)
    mg.mlp_setup(65536)
    mg.mlp_set_state(state, step)
    b = mg.rhs_fourier(seed=1_000_000 + 3)
    _, plain = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
    mg.set_local_solver("mlp_warm", "bf16")
    _, warm = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
    cg_plain = plain["cg_iterations"] / plain["local_solves"]
    cg_warm = warm["cg_iterations"] / warm["local_solves"]
    print(f"outer steps {plain['iterations']} / {warm['iterations']}, local CG per patch {cg_plain:.2f} / "
          f"{cg_warm:.2f}", flush=True)
    assert warm["converged"] and warm["rel_residual"] <= 1e-8
    assert warm["iterations"] == plain["iterations"]
    assert cg_warm <= 0.85 * cg_plain
    mg.set_local_solver("mlp", "bf16")
    mg.set_fallback(plain["history"][-1] ** (1.0 / plain["iterations"]))
    _, learned = mg.solve(b, rtol=1e-8, vcycle_dtype="f32", restart=10)
    print(f"learned in place of the local solve: {learned['iterations']} steps, fallback at "
          f"{learned['fallback_iteration']}", flush=True)
    assert learned["converged"] and learned["rel_residual"] <= 1e-8
    mg.set_local_solver("exact")
