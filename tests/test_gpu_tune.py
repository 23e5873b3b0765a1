"""Autotuner and launch plans on the GPU: tuned and forced plans change only how work is split,
so operators and solves stay within their parity bars of the FP64 oracle."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_autotune_plan_valid_and_cached(tmp_path):
    from paper_2602_09527_amd import api
    g = api.Geometry(256, 256, 360, 384, n_subsets=20)
    plan = api.autotune(g, reps=3, cache_path=str(tmp_path / "plans.json"))
    assert plan == g.get_plan()
    assert 1 <= plan["proj_split_full"] <= 64 and 1 <= plan["proj_split_subset"] <= 64
    assert 1 <= plan["bp_groups_full"] <= 16 and plan["bp_strip_subset"] in (1, 2, 4, 8)
    assert 2 <= plan["fgp_iters"] <= 16
    assert plan["bp_method_full"] in (1, 2) and plan["bp_method_subset"] in (1, 2)
    cache = json.load(open(tmp_path / "plans.json"))
    assert cache[g.key] == plan
    g2 = api.Geometry(256, 256, 360, 384, n_subsets=20)
    assert api.autotune(g2, cache_path=str(tmp_path / "plans.json")) == plan


@pytest.mark.parametrize("shape", [(64, 48, 30, 45, 4, 1, torch.float32), (37, 23, 29, 41, 4, 3, torch.float32),
                                   (60, 52, 45, 70, 5, 1, torch.float64)])
def test_autotune_odd_shapes(orc, shape):
    # sizes whose buffers are not multiples of the workspace alignment, a volume, FP64
    from paper_2602_09527_amd import api
    nx, ny, A, B, N, nz, dt = shape
    g = api.Geometry(nx, ny, A, B, n_subsets=N, nz=nz, dtype=dt)
    plan = api.autotune(g, reps=1)
    assert plan == g.get_plan()
    o = orc.Geometry(nx, ny, A, B, n_subsets=N, nz=nz)
    rng = np.random.default_rng(9)
    y = rng.standard_normal((nz, A, B))
    x = api.backproject(g, torch.from_numpy(y).to("cuda", dt), -1).cpu().numpy()
    assert _rel(x, orc.backproject(o, y, -1)) <= (1e-5 if dt == torch.float32 else 1e-12)


@pytest.mark.parametrize("plan", [
    dict(proj_split_full=1, proj_split_subset=1, bp_groups_full=1, bp_groups_subset=1,
         bp_strip_full=2, bp_strip_subset=1, fgp_iters=3, bp_method_full=2, bp_method_subset=1),
    dict(proj_split_full=16, proj_split_subset=12, bp_groups_full=16, bp_groups_subset=8,
         bp_strip_full=4, bp_strip_subset=8, fgp_iters=6, bp_method_full=1, bp_method_subset=2),
])
def test_forced_plans_keep_parity(orc, plan):
    from paper_2602_09527_amd import api
    nx, ny, A, B, N = 120, 100, 90, 160, 6
    g = api.Geometry(nx, ny, A, B, n_subsets=N)
    g.set_plan(plan)
    o = orc.Geometry(nx, ny, A, B, n_subsets=N)
    rng = np.random.default_rng(3)
    x = rng.random((1, ny, nx))
    y = rng.standard_normal((1, A, B))
    xt = torch.from_numpy(x).float().cuda()
    yt = torch.from_numpy(y).float().cuda()
    for subset in (-1, 2):
        ys = y if subset < 0 else y[:, subset::N]
        assert _rel(api.project(g, xt, subset).cpu().numpy(), orc.project(o, x, subset)) <= 1e-5
        assert _rel(api.backproject(g, torch.from_numpy(ys).float().cuda(), subset).cpu().numpy(),
                    orc.backproject(o, ys, subset)) <= 1e-5
    v = rng.random((1, ny, nx))
    d0 = np.zeros((2, 1, ny, nx))
    z_ref = orc.tv_prox_fgp(v, 0.05, 37, nonneg=True, dual=d0)
    dual = torch.zeros(g.dual_shape(), device="cuda")
    z = api.tv_prox(g, torch.from_numpy(v).float().cuda(), 0.05, 37, dual=dual)
    assert _rel(z.cpu().numpy(), z_ref) <= 1e-5


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-9)])
@pytest.mark.parametrize("rows,split,fused", [(2, 2, 1), (4, 4, 1), (2, 2, 2), (4, 4, 2)])
def test_gather_split_solve_matches_oracle(orc, dtype, tol, rows, split, fused):
    # the 128^2 solve (180 x 128, 10 subsets) with the pixel-driven backprojector whose waves
    # split the angles (its fused SVRG / ProxSkip update included), 10 epochs; the projector's
    # 4 partial sums per ray added by the reduction pass (fused = 1) or by the gather (2)
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.SMALL_2D
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed, with_phantom=False)
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, dtype=dtype)
    g.set_plan(dict(bp_method_full=2, bp_method_subset=2, bp_gather_rows=rows, bp_gather_split=split,
                    proj_split_subset=4, bp_gather_fused=fused))
    assert g.get_plan()["bp_gather_fused"] == fused
    o = orc.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
    L = json.load(open(__file__.replace("test_gpu_tune.py", "golden/lipschitz.json")))[w.key]["L"]
    kw = dict(gamma=1.0 / L, p=w.p, alpha=w.alpha, fgp_inner=w.fgp_inner, n_epochs=10,
              nonneg=True, seed=w.seed + 2)
    x, _, _, st = api.solve(g, torch.from_numpy(prob.b).to("cuda", dtype), api.SolverParams(**kw))
    xo, _, _, so, _ = orc.proxskip_svrg(o, prob.b, **kw)
    assert st["prox_calls"] == so["prox_calls"] > 0
    assert _rel(x.cpu().double().numpy(), xo) <= tol


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("estimator", ["svrg", "lsvrg", "saga"])
def test_gather_fused_same_bits(dtype, estimator):
    # the subset gather adding the projector's split partials itself gives the bits of the
    # reduction pass followed by the gather: uneven subsets (52 angles in 7), an odd split (a
    # ragged last pair of partials) and an even one, every estimator (SAGA subtracts b there)
    from paper_2602_09527_amd import api, synth
    nx, ny, A, B, N = 100, 90, 52, 150, 7
    prob = synth.make_problem(nx, ny, A, B, seed=3, with_phantom=False)
    g = api.Geometry(nx, ny, A, B, n_subsets=N, dtype=dtype)
    b = torch.from_numpy(prob.b).to("cuda", dtype)
    prm = api.SolverParams(gamma=1e-4, p=0.3, alpha=0.01, fgp_inner=20, n_epochs=3, seed=11,
                           estimator=estimator)
    _fused_against_reduction_pass(api, g, b, prm, (3, 2))


@pytest.mark.parametrize("estimator", ["svrg", "saga"])
def test_gather_fused_same_bits_volume(estimator):
    # the same on a 3-slice volume with 3D TV: every slice's partials and (SAGA) its rows of b
    from paper_2602_09527_amd import api
    nx, ny, nz, A, B, N = 100, 96, 3, 40, 150, 5
    rng = np.random.default_rng(8)
    g = api.Geometry(nx, ny, A, B, n_subsets=N, nz=nz)
    b = torch.from_numpy(rng.random((nz, A, B))).float().cuda()
    prm = api.SolverParams(gamma=1e-4, p=0.3, alpha=0.01, fgp_inner=10, n_epochs=2, seed=5,
                           estimator=estimator)
    _fused_against_reduction_pass(api, g, b, prm, (2, 3))


def _fused_against_reduction_pass(api, g, b, prm, splits):
    for psplit in splits:
        out = []
        for fused in (1, 2):
            g.set_plan(dict(bp_method_subset=2, proj_split_subset=psplit, bp_gather_fused=fused))
            assert (g.get_plan()["bp_gather_fused"], g.get_plan()["proj_split_subset"]) == (fused, psplit)
            x, h, dual, st = api.solve(g, b, prm)
            assert st["prox_calls"] > 0 and torch.isfinite(x).all()
            out.append((x, h, dual))
        for a, c in zip(*out):
            assert torch.equal(a, c)


def test_tuned_solve_matches_oracle(orc):
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.SMALL_2D
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed, with_phantom=False)
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
    api.autotune(g, reps=2)
    o = orc.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
    L = json.load(open(__file__.replace("test_gpu_tune.py", "golden/lipschitz.json")))[w.key]["L"]
    kw = dict(gamma=1.0 / L, p=w.p, alpha=w.alpha, fgp_inner=w.fgp_inner, n_epochs=10,
              nonneg=True, seed=w.seed + 2)
    xo, _, _, so, _ = orc.proxskip_svrg(o, prob.b, **kw)
    x, _, _, st = api.solve(g, torch.from_numpy(prob.b).float().cuda(), api.SolverParams(**kw))
    assert st["prox_calls"] == so["prox_calls"]
    assert _rel(x.cpu().numpy(), xo) <= 1e-4


TILES = [(4, 4), (4, 8), (8, 2), (8, 4), (8, 8), (16, 2), (16, 4)]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fgp_tiles_bitwise_equal(orc, dtype):
    # the tile shape, columns per lane and iterations per launch (up to 16 in FP32) decide only
    # which workgroup computes a pixel: every (tile, cols, T) gives the same bits, and those match
    # the FP64 oracle
    from paper_2602_09527_amd import api
    nx, ny = 150, 97   # several tiles of every shape, ragged in both directions
    g = api.Geometry(nx, ny, 30, 40, n_subsets=2, dtype=dtype)
    rng = np.random.default_rng(5)
    v = rng.random((1, ny, nx))
    d0 = 0.3 * rng.standard_normal((2, 1, ny, nx))
    vt = torch.from_numpy(v).to("cuda", dtype)
    ref = None
    for cols in (1, 2):
        for w, r in TILES:
            for T in (1, 3, 8) + ((12, 16) if dtype == torch.float32 else ()):
                g.set_plan(dict(fgp_waves=w, fgp_rows=r, fgp_iters=T, fgp_cols=cols))
                assert g.get_plan()["fgp_iters"] == min(T, w * r // 2 - 2)
                assert g.get_plan()["fgp_cols"] == cols
                dual = torch.from_numpy(d0).to("cuda", dtype)
                z = api.tv_prox(g, vt, 0.05, 29, dual=dual)
                torch.cuda.synchronize()
                if ref is None:
                    ref = (z.clone(), dual.clone())
                    z_ref = orc.tv_prox_fgp(v, 0.05, 29, nonneg=True, dual=d0.copy())
                    assert _rel(z.cpu().numpy(), z_ref) <= (1e-5 if dtype == torch.float32 else 1e-12)
                else:
                    assert torch.equal(z, ref[0]) and torch.equal(dual, ref[1]), (w, r, T, cols)


@pytest.mark.parametrize("shape", [(1, 40), (37, 1), (5, 3), (70, 2), (2, 65)])
def test_fgp_tiles_on_degenerate_images(orc, shape):
    # images narrower or shorter than one tile's halo: every tile and depth stays within the
    # image and matches the oracle
    from paper_2602_09527_amd import api
    nx, ny = shape
    g = api.Geometry(nx, ny, 8, 12, n_subsets=1)
    rng = np.random.default_rng(nx * 100 + ny)
    v = rng.random((1, ny, nx))
    z_ref = orc.tv_prox_fgp(v, 0.1, 23, nonneg=True, dual=np.zeros((2, 1, ny, nx)))
    vt = torch.from_numpy(v).to("cuda", torch.float32)
    for cols in (1, 2):
        for w, r in TILES:
            for T in (1, 8, 16):
                g.set_plan(dict(fgp_waves=w, fgp_rows=r, fgp_iters=T, fgp_cols=cols))
                z = api.tv_prox(g, vt, 0.1, 23, dual=torch.zeros(g.dual_shape(), device="cuda"))
                assert _rel(z.cpu().numpy(), z_ref) <= 1e-5, (w, r, T, cols)
