"""Serving loop on the GPU: requests of mixed sizes arrive while others run, are admitted by HBM
budget, and each result is bit for bit the result of solving that request alone (and of the
one-at-a-time baseline)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIDES = (64, 96, 128)
ANGLES = (30, 60, 90)
SUBSETS = {30: 5, 60: 6, 90: 10}


def _setup(n=12, rate=400.0):
    from paper_2602_09527_amd import serve
    trace = serve.make_trace(n, rate, seed=77, sides=SIDES, angles=ANGLES, subsets=SUBSETS)
    geoms = serve.GeometryCache("cuda", power_iters=20)
    geoms.warm(trace)
    bank = serve.data_bank(trace, "cuda")
    return trace, geoms, bank


def test_mix_equals_alone_and_sequential_bitwise():
    from paper_2602_09527_amd import serve
    trace, geoms, bank = _setup()
    cfg = serve.ServeConfig(fgp_inner=10, tol=2e-3, max_epochs=12, max_slots=5, steps_per_round=7)
    # a budget that holds about four of the mid-size requests forces queueing by memory
    sizes = sorted(serve.footprint_bytes(geoms.get(r)[0], serve.params_for(r, cfg, geoms.get(r)[1]))
                   for r in trace)
    cfg.budget_bytes = int(sum(sizes[len(sizes) // 2: len(sizes) // 2 + 4]))
    keep = {r.rid for r in trace[::3]}
    res, wall = serve.serve(trace, cfg, bank, geoms, keep=keep)
    assert len(res) == len(trace)
    for r in res:
        assert r["finished"] >= r["admitted"] >= 0 and r["latency"] > 0
        assert 1 <= r["epochs"] <= cfg.max_epochs
    seq, _ = serve.serve_sequential(trace, cfg, bank, geoms, keep=keep)
    by_rid = {r["rid"]: r for r in res}
    for s in seq:
        m = by_rid[s["rid"]]
        assert (s["epochs"], s["prox_calls"], s["last_rel_change"]) == \
            (m["epochs"], m["prox_calls"], m["last_rel_change"])
    for rid in sorted(keep):
        req = trace[rid]
        alone = serve.solve_alone(req, cfg, bank, geoms)
        assert torch.equal(by_rid[rid]["x"], alone), rid
        assert torch.equal({s["rid"]: s for s in seq}[rid]["x"], alone), rid
    summary = serve.summarize(res, wall)
    assert summary["requests"] == len(trace)


def test_requests_arriving_mid_run_are_admitted():
    # arrivals spread over time: later requests join while earlier ones are on the GPU
    from paper_2602_09527_amd import serve
    trace, geoms, bank = _setup(n=8, rate=500.0)
    cfg = serve.ServeConfig(fgp_inner=10, tol=1e-9, max_epochs=40, max_slots=8, steps_per_round=5)
    res, wall = serve.serve(trace, cfg, bank, geoms)
    overl = sum(1 for a in res for b in res
                if a["rid"] < b["rid"] and b["admitted"] < a["finished"])
    assert overl > 0
    assert all(r["epochs"] >= 1 for r in res)


def test_served_request_matches_the_oracle(orc):
    # a sampled request of a served mix, solved to the relative-change rule, against the FP64
    # oracle on the same data (its FP32 sinogram), step size and streams after the same epochs
    import numpy as np
    from paper_2602_09527_amd import serve
    trace, geoms, bank = _setup(n=6, rate=400.0)
    cfg = serve.ServeConfig(fgp_inner=20, tol=5e-3, max_epochs=40, max_slots=6, steps_per_round=7)
    pick = max(trace, key=lambda r: (r.side, r.n_angles))
    res, _ = serve.serve(trace, cfg, bank, geoms, keep={pick.rid})
    got = {r["rid"]: r for r in res}[pick.rid]
    assert got["converged"] and got["epochs"] < cfg.max_epochs
    g, L = geoms.get(pick)
    o = orc.Geometry(pick.side, pick.side, pick.n_angles, pick.n_bins, n_subsets=pick.n_subsets)
    b = bank[pick.rid].numpy().astype(np.float64)
    xo, _, _, so, relo = orc.proxskip_svrg(o, b, gamma=1.0 / L, p=cfg.p, alpha=cfg.alpha,
                                           fgp_inner=cfg.fgp_inner, n_epochs=got["epochs"],
                                           nonneg=True, seed=pick.seed + 2)
    assert so["prox_calls"] == got["prox_calls"]
    # the oracle crosses the tolerance at the same epoch end
    assert relo[-1] < cfg.tol * 1.01 and np.all(relo[:-1] >= cfg.tol * 0.99)
    x = got["x"].cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert rel <= 1e-4, rel
