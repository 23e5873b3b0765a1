"""Batched solves (solver_epochs over several handles): every problem of uneven size advances in
the same launches as the others, and its result is bit for bit the result of solving it alone.

The work-list kernels give each item its own geometry, buffers and launch plan, so an item's
arithmetic does not depend on what shares the launch; these tests hold the implementation to that.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem(nx, ny, A, B, N, seed, dtype, **kw):
    from paper_2602_09527_amd import api, synth
    prob = synth.make_problem(nx, ny, A, B, seed=seed, with_phantom=False)
    g = api.Geometry(nx, ny, A, B, n_subsets=N, dtype=dtype)
    b = torch.from_numpy(prob.b).to(device="cuda", dtype=dtype)
    L = api.lipschitz(g, 30)
    prm = dict(gamma=1.0 / L, p=0.2, alpha=0.01, fgp_inner=20, n_epochs=4, seed=seed + 2)
    prm.update(kw)
    return g, b, api.SolverParams(**prm)


MIX = [
    # nx, ny, A, B, N, seed, dtype, overrides
    (128, 128, 180, 128, 10, 11, torch.float32, {}),
    (96, 80, 90, 144, 5, 12, torch.float32, dict(p=0.5, fgp_inner=13)),
    (256, 256, 360, 384, 20, 13, torch.float32, dict(n_epochs=3)),
    (64, 64, 60, 96, 6, 14, torch.float64, dict(p=1.0, fgp_inner=7)),
    (120, 136, 72, 100, 8, 15, torch.float32, dict(plain_prox_svrg=True, p=1.0, fgp_inner=9)),
    (128, 128, 90, 192, 10, 16, torch.float32, dict(n_epochs=40, tol_rel_change=0.05)),
]


def _state(s):
    torch.cuda.synchronize()
    return s.x.clone(), s.h.clone(), s.dual.clone(), s.query()


def test_mixed_batch_bitwise_equals_alone():
    from paper_2602_09527_amd import api
    probs = [_problem(*m[:7], **m[7]) for m in MIX]
    alone = []
    for g, b, prm in probs:
        s = api.Solver(g, b, prm)
        s.epochs(prm.n_epochs)
        alone.append(_state(s))
    solvers = [api.Solver(g, b, prm) for g, b, prm in probs]
    api.run_epochs(solvers, max(p.n_epochs for _, _, p in probs))
    for k, s in enumerate(solvers):
        x, h, d, st = _state(s)
        xa, ha, da, sa = alone[k]
        assert st == sa, (k, st, sa)
        assert torch.equal(x, xa) and torch.equal(h, ha) and torch.equal(d, da), k
    # the tolerance handle stopped early, at the same epoch as alone
    assert 1 <= alone[-1][3]["epochs_done"] < 40


def test_many_slices_beyond_one_work_list():
    # 20 independent 64^2 slices (more items than one launch's work list holds)
    from paper_2602_09527_amd import api
    probs = [_problem(64, 64, 60, 96, 6, 100 + 3 * j, torch.float32, n_epochs=3) for j in range(20)]
    alone = []
    for g, b, prm in probs:
        s = api.Solver(g, b, prm)
        s.epochs(3)
        alone.append(_state(s))
    solvers = [api.Solver(g, b, prm) for g, b, prm in probs]
    api.run_epochs(solvers, 3)
    for k, s in enumerate(solvers):
        x, h, d, st = _state(s)
        assert st == alone[k][3]
        assert torch.equal(x, alone[k][0]) and torch.equal(h, alone[k][1]), k


def test_batch_member_matches_oracle(orc):
    # one member of a mixed batch against the FP64 oracle (1e-4 relative L2 after its epochs)
    from paper_2602_09527_amd import api, synth
    nx = ny = 96
    A, B, N = 120, 144, 8
    prob = synth.make_problem(nx, ny, A, B, seed=21, with_phantom=False)
    o = orc.Geometry(nx, ny, A, B, n_subsets=N)
    L = orc.lipschitz(o, 50)
    kw = dict(gamma=1.0 / L, p=0.25, alpha=0.01, fgp_inner=16, n_epochs=5, nonneg=True, seed=23)
    xo, _, _, so, _ = orc.proxskip_svrg(o, prob.b, **kw)
    g = api.Geometry(nx, ny, A, B, n_subsets=N)
    b = torch.from_numpy(prob.b).float().cuda()
    s = api.Solver(g, b, api.SolverParams(**kw))
    others = [api.Solver(*_problem(128, 96, 90, 160, 10, 30 + j, torch.float32)[:3]) for j in range(3)]
    api.run_epochs([others[0], s, others[1], others[2]], 5)
    st = s.query()
    assert st["prox_calls"] == so["prox_calls"]
    x = s.x.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-4


def test_batch_with_different_fgp_tiles_bitwise_equals_alone():
    # solves whose 2D TV prox runs on different tile shapes share rounds but not launches
    from paper_2602_09527_amd import api
    tiles = [(4, 8, 8, 1), (16, 2, 5, 2), (8, 8, 0, 2), (16, 4, 3, 1)]
    mix = [(128, 128, 180, 128, 10, 21, torch.float32, {}),
           (96, 80, 90, 144, 5, 22, torch.float32, dict(fgp_inner=13)),
           (150, 97, 72, 160, 8, 23, torch.float32, dict(p=0.5)),
           (64, 64, 60, 96, 6, 24, torch.float64, dict(fgp_inner=7))]
    probs = []
    for m, (w, r, t, cx) in zip(mix, tiles):
        g, b, prm = _problem(*m[:7], **m[7])
        g.set_plan(dict(g.get_plan(), fgp_waves=w, fgp_rows=r, fgp_iters=t, fgp_cols=cx))
        assert (g.get_plan()["fgp_waves"], g.get_plan()["fgp_rows"]) == (w, r)
        probs.append((g, b, prm))
    alone = []
    for g, b, prm in probs:
        s = api.Solver(g, b, prm)
        s.epochs(prm.n_epochs)
        alone.append(_state(s))
    solvers = [api.Solver(g, b, prm) for g, b, prm in probs]
    api.run_epochs(solvers, max(p.n_epochs for _, _, p in probs))
    for k, s in enumerate(solvers):
        x, h, d, st = _state(s)
        xa, ha, da, sa = alone[k]
        assert st == sa, (k, st, sa)
        assert torch.equal(x, xa) and torch.equal(h, ha) and torch.equal(d, da), k


def test_batch_gather_tall_tiles_bitwise_equals_alone():
    # a batch whose subset gathers fill the chip between them -- 12 x 128^2 on tiles of 2 rows per
    # wave with the angles split 4 ways: 12 x 3 x 64 = 2304 workgroups, at least the 2048 that
    # switch a batch to 4 rows per wave -- still gives every member the bits it gets alone, with
    # the projector's split partials added by the gather or by the reduction pass, FP32 and FP64
    from paper_2602_09527_amd import api
    probs = []
    for j in range(12):
        g, b, prm = _problem(128, 128, 180, 128, 10, 40 + j, torch.float64 if j == 5 else torch.float32,
                             n_epochs=2, p=0.3)
        g.set_plan(dict(bp_method_subset=2, bp_gather_rows=2, bp_gather_split=4, proj_split_subset=4,
                        bp_gather_fused=1 + j % 2))
        assert g.get_plan()["bp_gather_fused"] == 1 + j % 2
        probs.append((g, b, prm))
    alone = []
    for g, b, prm in probs:
        s = api.Solver(g, b, prm)
        s.epochs(prm.n_epochs)
        alone.append(_state(s))
    solvers = [api.Solver(g, b, prm) for g, b, prm in probs]
    api.run_epochs(solvers, 2)
    for k, s in enumerate(solvers):
        x, h, d, st = _state(s)
        xa, ha, da, sa = alone[k]
        assert st == sa, (k, st, sa)
        assert torch.equal(x, xa) and torch.equal(h, ha) and torch.equal(d, da), k
