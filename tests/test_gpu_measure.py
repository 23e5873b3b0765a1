"""Measurement support on the GPU: the library's per-launch HIP event timer counts the launches
of each kernel class inside a solve (and none captured into graphs), and kernel_time times one
kernel class alone.  Results of the solve are unchanged by the timer."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(epochs, **kw):
    from paper_2602_09527_amd import api, synth
    prob = synth.make_problem(96, 96, 120, 144, seed=8, with_phantom=False)
    g = api.Geometry(96, 96, 120, 144, n_subsets=10)
    g.set_plan(dict(bp_method_subset=1, bp_method_full=1, proj_split_subset=4, proj_split_full=2))
    b = torch.from_numpy(prob.b).to(device="cuda", dtype=torch.float32)
    prm = api.SolverParams(gamma=1.0 / api.lipschitz(g, 20), p=0.5, alpha=0.01, fgp_inner=10,
                           n_epochs=epochs, seed=3, **kw)
    return g, b, prm


def test_timer_counts_launches_and_leaves_results_alone():
    from paper_2602_09527_amd import api
    g, b, prm = _solver(3)
    ref = api.Solver(g, b, prm)
    ref.epochs(3)
    classes = ["backproject_subset", "backproject_full", "project_subset", "project_full",
               "backproject_combine", "project_reduce", "fgp2d"]
    s = api.Solver(g, b, prm)
    with api.KernelTimer(classes) as kt:
        s.epochs(3)
        torch.cuda.synchronize()
        res = {c: kt.result(c) for c in classes}
    assert torch.equal(s.x, ref.x) and torch.equal(s.h, ref.h)
    # per epoch: one snapshot (all angles) and 9 subset iterations, each split in two passes
    assert res["project_full"][1] == 3 and res["backproject_full"][1] == 3
    assert res["project_subset"][1] == 27 and res["backproject_subset"][1] == 27
    assert res["project_reduce"][1] == 30 and res["backproject_combine"][1] == 30
    assert res["fgp2d"][1] >= s.query()["prox_calls"] > 0
    for c in classes:
        ms, n = res[c]
        assert n == 0 or 0.0 < ms / n < 50.0, c


def test_graph_epochs_are_not_timed():
    from paper_2602_09527_amd import api
    g, b, prm = _solver(2)
    s = api.Solver(g, b, prm)
    with api.KernelTimer(["project_subset"]) as kt:
        s.epochs(2, graph=True)
        torch.cuda.synchronize()
        assert kt.result("project_subset")[1] == 0


def test_kernel_time_alone():
    from paper_2602_09527_amd import api, _native
    g, _, _ = _solver(1)
    for c in ("backproject_subset", "backproject_full", "project_subset", "project_full"):
        us = api.kernel_time(g, c, reps=20)
        assert 0.5 < us < 5e4, (c, us)
    with pytest.raises(_native.NativeError):   # the plan takes the scatter, not the gather
        api.kernel_time(g, "backproject_gather", reps=5)
