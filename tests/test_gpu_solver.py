"""GPU ProxSkip-SVRG (Algorithm 1, ProxSVRGSkip) against the FP64 oracle, through the C ABI.

Bars: the FP32 iterate within 1e-4 relative L2 of the oracle's after the fixed epochs; the FP64
instantiation within 1e-9; subset/coin streams bit-exact (prox-call counts equal); reductions
and resume/determinism properties bit for bit where the arithmetic makes them exact.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _L(w):
    return json.load(open(os.path.join(GOLDEN, "lipschitz.json")))[w.key]["L"]


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _setup(orc, w, dtype, n_epochs=None, **over):
    from paper_2602_09527_amd import api, synth
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed, nz=w.nz,
                              noise=w.noise, with_phantom=False)
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, nz=w.nz, dtype=dtype)
    o = orc.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, nz=w.nz)
    kw = dict(gamma=1.0 / _L(w), p=w.p, alpha=w.alpha, fgp_inner=w.fgp_inner,
              n_epochs=w.n_epochs if n_epochs is None else n_epochs, nonneg=w.nonneg,
              seed=w.seed + 2)
    kw.update(over)
    b_dev = torch.from_numpy(prob.b).to(device="cuda", dtype=dtype)
    return g, o, prob.b, b_dev, kw


def _gpu_run(g, b_dev, kw, **extra):
    from paper_2602_09527_amd import api
    prm = api.SolverParams(**{**kw, **extra})
    x, h, dual, st = api.solve(g, b_dev, prm)
    torch.cuda.synchronize()
    return x.cpu().numpy(), h.cpu().numpy(), dual.cpu().numpy(), st


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-9)])
def test_small_2d_30_epochs(orc, dtype, tol):
    # 128^2, 180 angles x 128 bins, 10 subsets, p = 0.1, 100 FGP iterations, 30 epochs
    from paper_2602_09527_amd import workloads
    w = workloads.SMALL_2D
    g, o, b, b_dev, kw = _setup(orc, w, dtype)
    xo, ho, do, so, relo = orc.proxskip_svrg(o, b, **kw)
    x, h, d, st = _gpu_run(g, b_dev, kw)
    assert st["epochs_done"] == so["epochs_done"] == 30
    assert st["iters_done"] == so["iters_done"] == 300
    assert st["prox_calls"] == so["prox_calls"]          # identical coin sequence
    assert _rel(x, xo) <= tol, _rel(x, xo)
    assert _rel(h, ho) <= 10 * tol, _rel(h, ho)
    assert abs(st["last_rel_change"] - so["last_rel_change"]) <= 10 * tol * so["last_rel_change"] + 1e-12


def test_single_2d_512_three_epochs(orc):
    # 512^2, 720 angles x 768 bins, 20 subsets (the benchmarked solve), 3 epochs
    from paper_2602_09527_amd import workloads
    w = workloads.SINGLE_2D
    g, o, b, b_dev, kw = _setup(orc, w, torch.float32, n_epochs=3)
    xo, _, _, so, _ = orc.proxskip_svrg(o, b, **kw)
    x, _, _, st = _gpu_run(g, b_dev, kw)
    assert st["prox_calls"] == so["prox_calls"]
    assert _rel(x, xo) <= 1e-4, _rel(x, xo)


def test_p1_equals_plain_prox_svrg(orc):
    # p = 1 reduces Algorithm 1 to proximal SVRG (ProxSVRG).
    from paper_2602_09527_amd import workloads
    w = workloads.SMALL_2D
    g, _, _, b_dev, kw = _setup(orc, w, torch.float32, n_epochs=4, p=1.0, fgp_inner=20)
    x1, _, _, s1 = _gpu_run(g, b_dev, kw)
    x2, h2, _, s2 = _gpu_run(g, b_dev, kw, plain_prox_svrg=True)
    assert s1["prox_calls"] == s2["prox_calls"] == 40
    assert np.array_equal(h2, np.zeros_like(h2))
    assert _rel(x1, x2) <= 1e-5


def test_trivial_prox_keeps_h_zero(orc):
    from paper_2602_09527_amd import workloads
    w = workloads.SMALL_2D
    g, o, b, b_dev, kw = _setup(orc, w, torch.float64, n_epochs=3, alpha=0.0, nonneg=False, p=0.3)
    x, h, _, st = _gpu_run(g, b_dev, kw)
    assert np.array_equal(h, np.zeros_like(h))
    xo, ho, _, so, _ = orc.proxskip_svrg(o, b, **kw)
    assert _rel(x, xo) <= 1e-12


def test_resume_and_determinism_bitwise(orc):
    from paper_2602_09527_amd import api, workloads
    w = workloads.SMALL_2D
    g, _, _, b_dev, kw = _setup(orc, w, torch.float32, n_epochs=4, fgp_inner=30)
    xa, ha, da, sa = _gpu_run(g, b_dev, kw)
    xb, hb, db, sb = _gpu_run(g, b_dev, kw)
    assert np.array_equal(xa, xb) and np.array_equal(ha, hb) and np.array_equal(da, db)
    # two epochs, then resume at k0 = 2N with the saved (x, h, dual)
    prm = api.SolverParams(**{**kw, "n_epochs": 2})
    x, h, dual, s1 = api.solve(g, b_dev, prm)
    prm2 = api.SolverParams(**{**kw, "n_epochs": 2, "k0": 2 * w.n_subsets})
    x, h, dual, s2 = api.solve(g, b_dev, prm2, x=x, h=h, dual=dual)
    assert np.array_equal(x.cpu().numpy(), xa) and np.array_equal(h.cpu().numpy(), ha)
    assert s1["prox_calls"] + s2["prox_calls"] == sa["prox_calls"]


def test_handles_and_tolerance(orc):
    from paper_2602_09527_amd import api, workloads
    w = workloads.SMALL_2D
    g, o, b, b_dev, kw = _setup(orc, w, torch.float32, n_epochs=40, fgp_inner=20, p=0.5)
    _, _, _, so, relo = orc.proxskip_svrg(o, b, **kw)
    tol = float(relo[12]) * 1.01
    first = int(np.argmax(relo < tol))
    s = api.Solver(g, b_dev, api.SolverParams(**{**kw, "tol_rel_change": tol}))
    s.epochs(100)
    st = s.query()
    assert st["epochs_done"] == first + 1
    assert abs(st["last_rel_change"] - relo[first]) <= 1e-3 * relo[first]
    # epoch-by-epoch calls equal one call
    s2 = api.Solver(g, b_dev, api.SolverParams(**kw))
    for _ in range(5):
        s2.epochs(1)
    s3 = api.Solver(g, b_dev, api.SolverParams(**kw))
    s3.epochs(5)
    torch.cuda.synchronize()
    assert torch.equal(s2.x, s3.x) and torch.equal(s2.h, s3.h)
    s3.cancel()
    with pytest.raises(Exception):
        s3.epochs(1)


def test_volume_3d_reduced_10_epochs(orc):
    # 8 slices of 128^2 coupled by 3D TV, 180 angles x 192 bins, 10 subsets, p = 0.05,
    # Poisson-log noise, 50 FGP iterations, 10 epochs (the volume workload at reduced size)
    from paper_2602_09527_amd import workloads
    w = workloads.VOLUME_3D_REDUCED
    g, o, b, b_dev, kw = _setup(orc, w, torch.float32)
    assert g.tv_dims == 3
    xo, ho, do, so, _ = orc.proxskip_svrg(o, b, **kw)
    x, h, d, st = _gpu_run(g, b_dev, kw)
    assert st["prox_calls"] == so["prox_calls"] > 0
    assert _rel(x, xo) <= 1e-4, _rel(x, xo)
    assert _rel(d, do) <= 1e-3, _rel(d, do)


@pytest.mark.parametrize("estimator", ["svrg", "lsvrg"])
def test_large_image_keeps_the_difference(orc, estimator):
    # 768^2: x and the snapshot outgrow one XCD's L2, so the solver keeps dx = x - xs for the
    # subset projector (written by the step's epilogue, or after a prox); p = 0.5 takes both paths
    from paper_2602_09527_amd import api, synth
    nx, A, B, N = 768, 180, 1024, 10
    prob = synth.make_problem(nx, nx, A, B, seed=61, with_phantom=False)
    g = api.Geometry(nx, nx, A, B, n_subsets=N)
    o = orc.Geometry(nx, nx, A, B, n_subsets=N)
    kw = dict(gamma=1.0 / api.lipschitz(g, 30), p=0.5, alpha=0.01, fgp_inner=20, n_epochs=2,
              nonneg=True, seed=62)
    xo, _, _, so, _ = orc.proxskip(o, prob.b, estimator=estimator, **kw)
    b = torch.from_numpy(prob.b).to(device="cuda", dtype=torch.float32)
    x, _, _, st = api.solve(g, b, api.SolverParams(estimator=estimator, **kw))
    torch.cuda.synchronize()
    assert st["prox_calls"] == so["prox_calls"] and st["prox_calls"] > 0
    assert _rel(x.cpu().numpy(), xo) <= 1e-4, _rel(x.cpu().numpy(), xo)
