"""Epochs issued as captured HIP graphs (solver_epochs_graph) give bit for bit the eager results,
on every replay, with eager work and synchronisations between the replays."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small(seed=101, **kw):
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.SMALL_2D
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=seed, with_phantom=False)
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
    L = json.load(open(os.path.join(GOLDEN, "lipschitz.json")))[w.key]["L"]
    prm = dict(gamma=1.0 / L, p=w.p, alpha=w.alpha, fgp_inner=30, n_epochs=6, seed=seed + 2)
    prm.update(kw)
    return g, torch.from_numpy(prob.b).float().cuda(), api.SolverParams(**prm)


def _state(s):
    torch.cuda.synchronize()
    return s.x.clone(), s.h.clone(), s.dual.clone(), s.query()


@pytest.mark.parametrize("plan", [None, dict(bp_method_subset=2, proj_split_subset=4, bp_gather_fused=2)])
def test_graph_replays_equal_eager_each_epoch(plan):
    # the automatic plan (scatter subsets), and the subset gather adding the projector's partials
    from paper_2602_09527_amd import api
    g, b, prm = _small(p=0.5)
    if plan:
        g.set_plan(plan)
        assert g.get_plan()["bp_gather_fused"] == 2
    eager = api.Solver(g, b, prm)
    ref = []
    for _ in range(6):
        eager.epochs(1)
        ref.append(_state(eager))
    gs = api.Solver(g, b, prm)
    junk = torch.zeros(1 << 20, device="cuda")
    for e in range(6):
        gs.epochs(1, graph=True)
        junk.add_(1.0)             # eager work between replays
        torch.cuda.synchronize()
        x, h, d, st = _state(gs)
        assert st == ref[e][3], e
        assert torch.equal(x, ref[e][0]) and torch.equal(h, ref[e][1]) and torch.equal(d, ref[e][2]), e


def test_graph_cache_reuse_with_fixed_topology():
    # p = 1: every epoch has the same coin pattern, so rounds after the first update one graph
    from paper_2602_09527_amd import api
    g, b, prm = _small(p=1.0, n_epochs=5)
    a = api.Solver(g, b, prm)
    a.epochs(5)
    c = api.Solver(g, b, prm)
    c.epochs(5, graph=True)
    xa, ha, da, sa = _state(a)
    xc, hc, dc, sc = _state(c)
    assert sa == sc and torch.equal(xa, xc) and torch.equal(ha, hc) and torch.equal(da, dc)


def test_graph_batched_mix_with_tolerance():
    from paper_2602_09527_amd import api
    probs = [_small(seed=101), _small(seed=111, p=0.3, fgp_inner=9),
             _small(seed=121, n_epochs=30, tol_rel_change=0.05)]
    eager = [api.Solver(*p) for p in probs]
    api.run_epochs(eager, 30)
    graph = [api.Solver(*p) for p in probs]
    api.run_epochs(graph, 30, graph=True)
    for k in range(3):
        xe, he, de, se = _state(eager[k])
        xg, hg, dg, sg = _state(graph[k])
        assert se == sg, k
        assert torch.equal(xe, xg) and torch.equal(he, hg) and torch.equal(de, dg), k
    assert eager[2].query()["epochs_done"] < 30


def test_graph_refuses_mid_epoch_handles():
    from paper_2602_09527_amd import api, _native
    g, b, prm = _small()
    s = api.Solver(g, b, prm)
    api.run_steps([s], 3)
    with pytest.raises(_native.NativeError):
        s.epochs(1, graph=True)
    api.run_steps([s], 7)          # back at an epoch start (N = 10)
    s.epochs(1, graph=True)
    assert s.query()["epochs_done"] == 2
