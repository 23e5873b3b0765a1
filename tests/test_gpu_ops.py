"""GPU parity of the projector, backprojector and FGP TV prox against the FP64 oracle, through
the C ABI (HIP path only).

Bars: FP32 kernels within 1e-5 relative L2 of the oracle; the FP64 instantiation within 1e-12
(projector, backprojector) and 1e-11 (FGP, whose dual step 1/(8 tau) amplifies rounding).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (nx, ny, nz, A, B, N, du, off): configs' shapes plus ragged ones (odd sizes, several tiles
# with a ragged tail, nz > 1, A not divisible by N, bins finer/coarser than pixels).
SHAPES = [
    (128, 128, 1, 180, 128, 10, 1.0, 0.0),     # 128^2 image, 180 x 128 sinogram, 10 subsets
    (37, 23, 1, 29, 41, 4, 0.7, 0.3),
    (64, 48, 3, 90, 97, 7, 1.3, -0.45),
    (1, 1, 1, 3, 2, 1, 1.0, 0.0),
    (200, 70, 2, 45, 260, 5, 1.0, 0.5),
]


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _pair(orc, shape, dtype):
    from paper_2602_09527_amd import api
    nx, ny, nz, A, B, N, du, off = shape
    g = api.Geometry(nx, ny, A, B, n_subsets=N, nz=nz, bin_width=du, det_offset=off, dtype=dtype)
    o = orc.Geometry(nx, ny, A, B, n_subsets=N, nz=nz, du=du, off=off)
    return g, o


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-12)])
@pytest.mark.parametrize("shape", SHAPES)
def test_project_parity(orc, shape, dtype, tol):
    from paper_2602_09527_amd import api
    g, o = _pair(orc, shape, dtype)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, g.image_shape) + 0.1 * rng.standard_normal(g.image_shape)
    xd = _dev(x, dtype)
    for subset in [-1] + list(range(g.n_subsets)):
        y = api.project(g, xd, subset).cpu().numpy()
        yo = orc.project(o, x, subset)
        assert y.shape == yo.shape
        assert _rel(y, yo) <= tol, (subset, _rel(y, yo))


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-12)])
@pytest.mark.parametrize("shape", SHAPES)
def test_backproject_parity(orc, shape, dtype, tol):
    from paper_2602_09527_amd import api
    g, o = _pair(orc, shape, dtype)
    rng = np.random.default_rng(12)
    for subset in [-1] + list(range(g.n_subsets)):
        y = rng.standard_normal(g.sino_shape(subset))
        x = api.backproject(g, _dev(y, dtype), subset).cpu().numpy()
        xo = orc.backproject(o, y, subset)
        assert _rel(x, xo) <= tol, (subset, _rel(x, xo))
    # accumulate adds onto the existing image
    y = rng.standard_normal(g.sino_shape(0))
    base = rng.standard_normal(g.image_shape)
    out = _dev(base, dtype)
    api.backproject(g, _dev(y, dtype), 0, out=out, accumulate=True)
    assert _rel(out.cpu().numpy(), base + orc.backproject(o, y, 0)) <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 2e-6), (torch.float64, 1e-13)])
def test_dot_test_on_gpu(orc, dtype, tol):
    from paper_2602_09527_amd import api
    g, _ = _pair(orc, (96, 80, 2, 64, 130, 4, 1.0, 0.2), dtype)
    rng = np.random.default_rng(13)
    for subset in (-1, 0, 3):
        x = _dev(rng.standard_normal(g.image_shape), dtype)
        y = _dev(rng.standard_normal(g.sino_shape(subset)), dtype)
        lhs = float(torch.sum(api.project(g, x, subset).double() * y.double()))
        rhs = float(torch.sum(x.double() * api.backproject(g, y, subset).double()))
        assert abs(lhs - rhs) <= tol * (abs(lhs) + abs(rhs))


def test_operators_full_size_512(orc):
    # 512^2 image, 720 angles x 768 bins, 20 subsets: whole outputs against the oracle.
    from paper_2602_09527_amd import api, synth
    g, o = _pair(orc, (512, 512, 1, 720, 768, 20, 1.0, 0.0), torch.float32)
    x = synth.rasterize(synth.random_ellipses(202, 10), 512, 512)
    xd = _dev(x, torch.float32)
    for subset in (-1, 0, 13):
        assert _rel(api.project(g, xd, subset).cpu().numpy(), orc.project(o, x, subset)) <= 1e-5
    rng = np.random.default_rng(14)
    for subset in (-1, 7):
        y = rng.standard_normal(g.sino_shape(subset))
        assert _rel(api.backproject(g, _dev(y, torch.float32), subset).cpu().numpy(),
                    orc.backproject(o, y, subset)) <= 1e-5


def test_repeat_runs_bitwise(orc):
    from paper_2602_09527_amd import api
    g, _ = _pair(orc, SHAPES[2], torch.float32)
    rng = np.random.default_rng(15)
    x = _dev(rng.standard_normal(g.image_shape), torch.float32)
    y = _dev(rng.standard_normal(g.sino_shape(-1)), torch.float32)
    a1, a2 = api.project(g, x), api.project(g, x)
    b1, b2 = api.backproject(g, y), api.backproject(g, y)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


# ---------------------------------------------------------------------------------------------
# TV prox (FGP)
# ---------------------------------------------------------------------------------------------

PROX_SHAPES = [(128, 128, 1), (37, 23, 1), (70, 33, 1), (1, 1, 1), (24, 20, 4), (9, 7, 3)]


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-11)])
@pytest.mark.parametrize("shape", PROX_SHAPES)
@pytest.mark.parametrize("n_inner", [0, 1, 7, 8, 9, 50])
def test_tv_prox_parity(orc, shape, dtype, tol, n_inner):
    from paper_2602_09527_amd import api
    nx, ny, nz = shape
    g = api.Geometry(nx, ny, 4, 8, nz=nz, dtype=dtype)
    rng = np.random.default_rng(16 + n_inner)
    v = rng.uniform(-0.2, 1.0, g.image_shape)
    dual0 = rng.uniform(-0.6, 0.6, g.dual_shape())
    for nonneg in (False, True):
        for tau in (1e-3, 0.05, 0.4):
            d_o = dual0.copy()
            zo = orc.tv_prox_fgp(v, tau, n_inner, nonneg=nonneg, dual=d_o)
            d_g = _dev(dual0, dtype)
            z = api.tv_prox(g, _dev(v, dtype), tau, n_inner, nonneg=nonneg, dual=d_g)
            assert _rel(z.cpu().numpy(), zo) <= tol, (nonneg, tau, _rel(z.cpu().numpy(), zo))
            assert _rel(d_g.cpu().numpy(), d_o) <= 10 * tol


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_tv_prox_cold_start_alias_and_tau0(orc, dtype):
    from paper_2602_09527_amd import api
    g = api.Geometry(53, 41, 4, 8, dtype=dtype)
    rng = np.random.default_rng(17)
    v = rng.uniform(-0.3, 1.0, g.image_shape)
    zo = orc.tv_prox_fgp(v, 0.1, 20, nonneg=True)
    vd = _dev(v, dtype)
    z = api.tv_prox(g, vd, 0.1, 20, nonneg=True, dual=None, out=vd)   # z aliases v, cold start
    tol = 1e-5 if dtype == torch.float32 else 1e-11
    assert z.data_ptr() == vd.data_ptr()
    assert _rel(z.cpu().numpy(), zo) <= tol
    # tau = 0: projection onto C (or identity), dual untouched
    dual = _dev(rng.standard_normal(g.dual_shape()), dtype)
    d0 = dual.clone()
    z0 = api.tv_prox(g, _dev(v, dtype), 0.0, 10, nonneg=True, dual=dual)
    assert torch.equal(z0.cpu(), torch.from_numpy(np.maximum(v, 0.0)).to(dtype))
    assert torch.equal(dual, d0)
    z1 = api.tv_prox(g, _dev(v, dtype), 0.0, 10, nonneg=False)
    assert torch.equal(z1.cpu(), torch.from_numpy(v).to(dtype))


def test_tv_prox_full_size_512(orc):
    from paper_2602_09527_amd import api, synth
    g = api.Geometry(512, 512, 4, 8)
    v = synth.rasterize(synth.random_ellipses(3, 10), 512, 512)
    v = v + 0.05 * np.random.default_rng(18).standard_normal(v.shape)
    dual = np.zeros((2, 1, 512, 512))
    zo = orc.tv_prox_fgp(v, 2e-3, 50, nonneg=True, dual=dual)
    dg = torch.zeros(g.dual_shape(), device="cuda")
    z = api.tv_prox(g, _dev(v, torch.float32), 2e-3, 50, nonneg=True, dual=dg)
    assert _rel(z.cpu().numpy(), zo) <= 1e-5


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-12)])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("method,rows,split", [(1, 0, 0), (2, 0, 0), (2, 2, 2), (2, 4, 2), (2, 2, 4),
                                               (2, 4, 4)])
def test_backproject_methods_parity(orc, shape, dtype, tol, method, rows, split):
    # both backprojector methods forced for all angles and for subsets (the gather applies where
    # adjacent rays are at least one pixel apart; elsewhere the scatter serves the call), the
    # gather with its tiles' rows per wave and angle split
    from paper_2602_09527_amd import api
    g, o = _pair(orc, shape, dtype)
    g.set_plan(dict(bp_method_full=method, bp_method_subset=method, bp_gather_rows=rows,
                    bp_gather_split=split))
    rng = np.random.default_rng(40 + method)
    for subset in [-1] + list(range(g.n_subsets)):
        y = rng.standard_normal(g.sino_shape(subset))
        x = api.backproject(g, _dev(y, dtype), subset).cpu().numpy()
        assert _rel(x, orc.backproject(o, y, subset)) <= tol, (subset, method)


def test_strided_buffers_are_refused_not_copied():
    # an in/out buffer given as a strided view must raise: a reshaped copy would receive the
    # result (or the warm-start dual) instead of the caller's tensor
    from paper_2602_09527_amd import api
    g = api.Geometry(16, 16, 12, 16, n_subsets=2)
    v = torch.rand(g.image_shape, device="cuda")
    dual_big = torch.zeros((2, 1, 16, 32), device="cuda")
    with pytest.raises(ValueError):
        api.tv_prox(g, v, 0.1, 5, dual=dual_big[..., ::2])
    with pytest.raises(ValueError):
        api.project(g, torch.rand(1, 16, 32, device="cuda")[..., ::2])
    # a contiguous tensor of another shape with the right count is a view: results land in it
    flat = torch.zeros(2 * 16 * 16, device="cuda")
    api.tv_prox(g, v, 0.1, 5, dual=flat)
    torch.cuda.synchronize()
    assert float(flat.abs().sum()) > 0


def test_device_alloc_workspace():
    """A workspace from device_alloc (physically contiguous when the driver can provide it) gives
    the same bits as one from torch; workspaces of CONTIGUOUS_MIN_BYTES and more come from it."""
    from paper_2602_09527_amd import api
    g = api.Geometry(61, 13, 20, 30, nz=5)
    gen = torch.Generator(device="cuda").manual_seed(5)
    v = torch.rand(g.image_shape, device="cuda", generator=gen)
    nbytes = g.lib.tv_prox_workspace_bytes(g.handle)
    outs = []
    for ws in (torch.empty(nbytes, dtype=torch.uint8, device="cuda"), api.DeviceBuffer(nbytes, g.device)):
        g._ws = {"fgp": ws}
        dual = torch.zeros(g.dual_shape(), device="cuda")
        outs.append((api.tv_prox(g, v, 0.05, 9, dual=dual), dual))
        torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    buf = g._ws["fgp"]
    assert isinstance(buf.contiguous, bool) and buf.numel() == nbytes
    g._ws = {}
    del buf   # device_free waits for the queued work, then frees
    small = api.workspace_buffer(1 << 20, g.device)
    assert isinstance(small, torch.Tensor) and small.numel() == 1 << 20
    big = api.workspace_buffer(api.CONTIGUOUS_MIN_BYTES, g.device)
    assert isinstance(big, api.DeviceBuffer) and big.numel() == api.CONTIGUOUS_MIN_BYTES
    del big


def test_solver_with_device_alloc_workspaces(monkeypatch):
    """Every workspace of a solve, a prox and an autotune taken from device_alloc (the threshold
    lowered so that a small problem uses it) gives the same bits as torch workspaces."""
    from paper_2602_09527_amd import api, synth
    prob = synth.make_problem(96, 96, 60, 140, seed=4, with_phantom=False)
    b = torch.from_numpy(prob.b).float().cuda()
    runs = []
    for threshold in (1 << 62, 1):
        monkeypatch.setattr(api, "CONTIGUOUS_MIN_BYTES", threshold)
        g = api.Geometry(96, 96, 60, 140, n_subsets=6)
        api.autotune(g, reps=1, store=False)          # its workspace too; then one fixed plan
        g.set_plan(dict(proj_split_full=2, proj_split_subset=3, bp_method_subset=2))
        s = api.Solver(g, b, api.SolverParams(gamma=1.0 / 4000.0, p=0.5, alpha=0.01, fgp_inner=9,
                                              n_epochs=3, seed=2))
        assert isinstance(s.ws, api.DeviceBuffer) == (threshold == 1)
        s.epochs(3)
        dual = torch.zeros(g.dual_shape(), device="cuda")
        z = api.tv_prox(g, s.x, 0.02, 7, dual=dual)
        torch.cuda.synchronize()
        runs.append((s.x.clone(), s.h.clone(), z.clone(), dual.clone(), g.get_plan()))
        del s
    (xa, ha, za, da, pa), (xb, hb, zb, db, pb) = runs
    assert pa == pb
    assert torch.equal(xa, xb) and torch.equal(ha, hb) and torch.equal(za, zb) and torch.equal(da, db)


@pytest.mark.parametrize("shape", [(97, 131, 2, 77, 211, 6, 1.3, 0.45), (200, 70, 1, 45, 260, 5, 1.0, -2.5),
                                   (300, 300, 1, 361, 500, 19, 1.7, 0.0), (128, 128, 1, 180, 128, 10, 1.0, 0.0)])
def test_gather_matches_scatter_pixelwise(shape):
    # the gather's ray search and walks against the scatter, pixel by pixel: a ray missed or
    # taken twice at one pixel moves that pixel by about |y| / |.|, far beyond the max-norm bar,
    # while an L2 bar over the image could hide it
    from paper_2602_09527_amd import api
    nx, ny, nz, A, B, N, bw, off = shape
    g = api.Geometry(nx, ny, A, B, n_subsets=N, nz=nz, bin_width=bw, det_offset=off)
    gen = torch.Generator(device="cuda").manual_seed(nx + A)
    for subset in (-1, 0, N // 2):
        y = torch.randn(g.sino_shape(subset), device="cuda", generator=gen)
        g.set_plan(dict(bp_method_full=1, bp_method_subset=1))
        ref = api.backproject(g, y, subset).double()
        for rows in (2, 4):
            g.set_plan(dict(bp_method_full=2, bp_method_subset=2, bp_gather_rows=rows, bp_gather_split=1))
            got = api.backproject(g, y, subset).double()
            err = float((got - ref).abs().max())
            assert err <= 1e-5 * float(ref.abs().max()), (subset, rows, err)
