"""ProjectSubset (torch.autograd.Function): gradients by central finite differences and the
dot-product test on a batch of 64 images of 256^2 (360 angles x 384 bins), gradcheck in FP64 on
a small shape, and the backward pass against the FP64 oracle's adjoint."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def batch():
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.AUTOGRAD_BATCH
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, nz=w.nz)
    x = torch.from_numpy(synth.perturbed_batch(w.nz, w.nx, w.ny, seed=w.seed)).float().cuda()
    return g, x


def _loss64(y, target):
    return 0.5 * float(torch.sum((y.double() - target.double()) ** 2))


def test_finite_differences_batch64(batch):
    # Central differences with eps = 1e-3 along 8 seeded directions of the loss
    # l(x) = 1/2 ||A x - t||^2.  The loss is quadratic, so the difference quotient is exact up to
    # rounding; in FP32 that rounding grows as 1/eps (the projections of x +- eps v differ in their
    # last bits), so the eps = 1e-3 quotient is taken with the FP64 instantiation of the same
    # projector, and the FP32 backward pass is checked against it.  An FP32 quotient at eps = 0.1
    # checks the FP32 pair end to end.
    from paper_2602_09527_amd import api
    from paper_2602_09527_amd.autograd import ProjectSubset
    g, x = batch
    g64 = api.Geometry(g.nx, g.ny, g.n_angles, g.n_bins, nz=g.nz, dtype=torch.float64)
    gen = torch.Generator(device="cuda").manual_seed(5)
    target = torch.randn(g.sino_shape(-1), device="cuda", generator=gen) * 10.0
    grads = {}
    for geom, dt in ((g, torch.float32), (g64, torch.float64)):
        xr = x.to(dt).clone().requires_grad_(True)
        y = ProjectSubset.apply(xr, geom, -1)
        (0.5 * torch.sum((y - target.to(dt)) ** 2)).backward()
        grads[dt] = xr.grad.double()
    x64 = x.double()
    for k in range(8):
        v = torch.randn(x.shape, device="cuda", generator=gen, dtype=torch.float64)
        eps = 1e-3
        fd = (_loss64(ProjectSubset.apply(x64 + eps * v, g64, -1), target)
              - _loss64(ProjectSubset.apply(x64 - eps * v, g64, -1), target)) / (2 * eps)
        an64 = float(torch.sum(grads[torch.float64] * v))
        an32 = float(torch.sum(grads[torch.float32] * v))
        assert abs(fd - an64) <= 1e-7 * abs(an64), (k, fd, an64)
        assert abs(fd - an32) <= 1e-5 * abs(an64), (k, fd, an32)
        if k < 2:
            v32 = v.float()
            e = 0.1
            fd32 = (_loss64(ProjectSubset.apply(x + e * v32, g, -1), target)
                    - _loss64(ProjectSubset.apply(x - e * v32, g, -1), target)) / (2 * e)
            assert abs(fd32 - an32) <= 1e-3 * abs(an32), (k, fd32, an32)


def test_dot_product_batch64(batch):
    from paper_2602_09527_amd import api
    g, x = batch
    gen = torch.Generator(device="cuda").manual_seed(6)
    y = torch.randn(g.sino_shape(-1), device="cuda", generator=gen)
    lhs = float(torch.sum(api.project(g, x).double() * y.double()))
    rhs = float(torch.sum(x.double() * api.backproject(g, y).double()))
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs))


def test_subset_autograd_matches_oracle_adjoint(orc):
    from paper_2602_09527_amd import api
    from paper_2602_09527_amd.autograd import ProjectSubset
    g = api.Geometry(48, 40, 30, 64, n_subsets=3, nz=3)
    o = orc.Geometry(48, 40, 30, 64, n_subsets=3, nz=3)
    rng = np.random.default_rng(7)
    x = torch.from_numpy(rng.standard_normal((3, 40, 48))).float().cuda().requires_grad_(True)
    gy = rng.standard_normal(g.sino_shape(1))
    y = ProjectSubset.apply(x, g, 1)
    y.backward(torch.from_numpy(gy).float().cuda())
    ref = orc.backproject(o, gy, 1)
    got = x.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def test_gradcheck_fp64():
    from paper_2602_09527_amd import api
    from paper_2602_09527_amd.autograd import ProjectSubset
    g = api.Geometry(8, 7, 6, 11, n_subsets=2, nz=2, det_offset=0.3, dtype=torch.float64)
    x = torch.randn(g.image_shape, dtype=torch.float64, device="cuda", requires_grad=True)
    for subset in (-1, 0, 1):
        assert torch.autograd.gradcheck(lambda t: ProjectSubset.apply(t, g, subset), (x,),
                                        eps=1e-6, atol=1e-8, rtol=1e-6)
