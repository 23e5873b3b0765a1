"""Host logic of the serving loop: the request trace and first-come-first-served admission by
HBM budget and slot count (no GPU)."""
import numpy as np
import pytest

from paper_2602_09527_amd import serve, workloads


def test_trace_is_seeded_and_shaped():
    a = serve.make_trace(400, 20.0, seed=505)
    b = serve.make_trace(400, 20.0, seed=505)
    assert a == b
    assert [r.rid for r in a] == list(range(400))
    t = np.array([r.arrival for r in a])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    # mean gap 1/20 s (exponential gaps: the mean of 399 gaps is within 20% with high probability)
    assert abs(np.mean(np.diff(t)) - 0.05) < 0.01
    assert {r.side for r in a} == set(workloads.SERVE_SIDES)
    assert {r.n_angles for r in a} == set(workloads.SERVE_ANGLES)
    for r in a:
        assert r.n_bins == 3 * r.side // 2
        assert r.n_subsets == workloads.SERVE_SUBSETS[r.n_angles]
    assert len({r.seed for r in a}) == 400
    assert serve.make_trace(400, 20.0, seed=506) != a


def _req(rid, t):
    return serve.Request(rid, t, 64, 30, 96, 5, rid)


def test_admission_fifo_budget_and_slots():
    cfg = serve.ServeConfig(budget_bytes=100, max_slots=3)
    size = {0: 40, 1: 40, 2: 30, 3: 10, 4: 10}
    q = [_req(i, 0.1 * i) for i in range(5)]
    sz = lambda r: size[r.rid]
    # nothing has arrived before t = 0
    assert serve.admit(q, 0, 0, -1.0, cfg, sz) == []
    # at t = 0.15 requests 0 and 1 have arrived and fit (80 <= 100)
    assert [r.rid for r in serve.admit(q, 0, 0, 0.15, cfg, sz)] == [0, 1]
    # at t = 1: request 2 (30) would exceed the budget after 0 and 1, and blocks 3 and 4 behind it
    assert [r.rid for r in serve.admit(q, 0, 0, 1.0, cfg, sz)] == [0, 1]
    # with 50 bytes in use, only request 0 fits
    assert [r.rid for r in serve.admit(q, 50, 1, 1.0, cfg, sz)] == [0]
    # slot cap
    cfg2 = serve.ServeConfig(budget_bytes=10**9, max_slots=3)
    assert [r.rid for r in serve.admit(q, 0, 1, 1.0, cfg2, sz)] == [0, 1]
    # a request larger than the whole budget cannot ever be served
    cfg3 = serve.ServeConfig(budget_bytes=20, max_slots=3)
    with pytest.raises(ValueError):
        serve.admit(q, 0, 0, 1.0, cfg3, sz)
