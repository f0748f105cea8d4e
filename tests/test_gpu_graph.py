"""Graph replay of the CG check windows and the autotuner of the Krylov step's
launch parameters (GPU)."""
import numpy as np
import pytest
import torch

from paper_2412_19207_amd import binding
from paper_2412_19207_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()


@pytest.mark.parametrize("k,precision", [(1, "fp64"), (3, "fp64"), (32, "mixed")])
def test_graph_replays_match_eager_launches(k, precision):
    """Several solves (each replaying its captured windows many times) and an
    adjoint solve, with eager work and synchronisations between them: every
    result is bitwise the one of eager launches."""
    _need_gpu()
    prob = wl.small2d(k=k)
    F = torch.as_tensor(prob.F, device=DEV)
    out = {}
    for graph in [0, 1]:
        s = binding.Solver(prob, device=DEV, precision=precision)
        s.pca(1e-10)
        s.set_tuning(use_graph=graph)
        res = []
        for rep in range(3):
            W, info = s.solve(F, tol=1e-12, maxiter=3000, check_every=10)
            assert info["status"] == 0
            z = s.apply_precond(W)  # eager work between the replays
            torch.cuda.synchronize()
            res.append((W.clone(), info["rhs_iterations"].copy(), z))
        dF, st = s.solve_backward(W, tol=1e-12, maxiter=3000)
        assert st["status"] == 0
        res.append((dF, None, None))
        n_graphs, failed = s.graph_state()
        assert failed == 0
        assert (n_graphs > 0) == bool(graph), n_graphs
        out[graph] = res
        s.close()
    for (We, ie, ze), (Wg, ig, zg) in zip(out[0], out[1]):
        assert torch.equal(We, Wg)
        if ie is not None:
            assert np.array_equal(ie, ig)
            assert torch.equal(ze, zg)


def test_autotune_picks_valid_parameters(tmp_path, monkeypatch):
    """The autotuner returns parameters in their ranges, the handle keeps them,
    the cache returns them again, and the solution agrees with the default
    parameters' to rounding."""
    _need_gpu()
    monkeypatch.setenv("RANN_DD_TUNING_CACHE", str(tmp_path / "tuning.json"))
    prob = wl.small2d(k=1)
    F = torch.as_tensor(prob.F, device=DEV)
    s0 = binding.Solver(prob, device=DEV)
    s0.pca(1e-10)
    W0, _ = s0.solve(F, tol=1e-12, maxiter=3000)
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10)
    rec = s.autotune(1, iters=10)
    assert rec["source"] == "timed" and rec["us_per_iteration"] > 0
    t = s.tuning()
    assert t == {k: rec[k] for k in ("tile_grid", "red_cap", "use_graph")}
    assert t["tile_grid"] in (256, 512, 768, 1024) and t["red_cap"] in (64, 128, 240)
    W, info = s.solve(F, tol=1e-12, maxiter=3000)
    assert info["status"] == 0
    assert float((W - W0).norm() / W0.norm()) <= 1e-10
    s2 = binding.Solver(prob, device=DEV)
    s2.pca(1e-10)
    rec2 = s2.autotune(1, iters=10)
    assert rec2["source"] == "cache" and s2.tuning() == t
    for x in (s0, s, s2):
        x.close()
