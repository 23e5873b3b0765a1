"""The reference solver x* (preconditioned PDHG for Eq. 5) on the GPU against the FP64 oracle,
through the C ABI: FP32 within 1e-4 relative L2 after the same iterations, FP64 within 1e-9;
continuing a run from its state (x, y1, y2) is bit for bit one longer run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _problem(nx, A, B, seed, dtype):
    from paper_2602_09527_amd import api, synth
    prob = synth.make_problem(nx, nx, A, B, seed=seed, with_phantom=False)
    g = api.Geometry(nx, nx, A, B, n_subsets=1, dtype=dtype)
    return g, prob.b, torch.from_numpy(prob.b).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-9)])
@pytest.mark.parametrize("nonneg", [True, False])
def test_pdhg_against_oracle(orc, dtype, tol, nonneg):
    from paper_2602_09527_amd import api
    nx, A, B, K = 64, 90, 96, 300
    g, b, b_dev = _problem(nx, A, B, 51, dtype)
    o = orc.Geometry(nx, nx, A, B, n_subsets=1)
    xo, y1o, y2o = orc.pdhg(o, b, alpha=0.05, n_iters=K, nonneg=nonneg)
    x, y1, y2 = api.pdhg(g, b_dev, alpha=0.05, n_iters=K, nonneg=nonneg)
    torch.cuda.synchronize()
    assert _rel(x.cpu().numpy(), xo) <= tol, _rel(x.cpu().numpy(), xo)
    assert _rel(y1.cpu().numpy(), y1o) <= tol, _rel(y1.cpu().numpy(), y1o)
    assert _rel(y2.cpu().numpy(), y2o) <= 10 * tol, _rel(y2.cpu().numpy(), y2o)


def test_pdhg_volume_against_oracle(orc):
    # 3D TV couples the slices: 4 x 48^2
    from paper_2602_09527_amd import api, synth
    nx, nz, A, B, K = 48, 4, 60, 72, 200
    prob = synth.make_problem(nx, nx, A, B, seed=52, nz=nz, with_phantom=False)
    g = api.Geometry(nx, nx, A, B, n_subsets=1, nz=nz, dtype=torch.float64)
    o = orc.Geometry(nx, nx, A, B, n_subsets=1, nz=nz)
    xo, _, _ = orc.pdhg(o, prob.b, alpha=0.05, n_iters=K)
    x, _, _ = api.pdhg(g, torch.from_numpy(prob.b).cuda(), alpha=0.05, n_iters=K)
    torch.cuda.synchronize()
    assert _rel(x.cpu().numpy(), xo) <= 1e-9, _rel(x.cpu().numpy(), xo)


def test_pdhg_continuation_bitwise():
    from paper_2602_09527_amd import api
    g, _, b = _problem(96, 120, 144, 53, torch.float32)
    x1, y11, y21 = api.pdhg(g, b, alpha=0.02, n_iters=120)
    x2, y12, y22 = api.pdhg(g, b, alpha=0.02, n_iters=50)
    api.pdhg(g, b, alpha=0.02, n_iters=70, x=x2, y1=y12, y2=y22)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and torch.equal(y11, y12) and torch.equal(y21, y22)
