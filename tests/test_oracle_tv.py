"""Pins of the oracle's isotropic TV and its FGP proximal operator (no GPU).

prox_{tau (TV + I_C)}(v) = argmin_z 1/2 ||z - v||^2 + tau TV(z) + I_C(z)  (Eq. 3 with the
regulariser of Eq. 5), computed by FGP (Beck & Teboulle 2009) as the paper prescribes (Sec. 2.1).
"""
import numpy as np
import pytest


def _D(z):
    """Forward differences with a zero last difference, written independently of the oracle."""
    z = np.asarray(z, dtype=float)
    out = []
    for ax in range(z.ndim - 1, -1, -1):   # x (last axis) first, then y, then z
        d = np.zeros_like(z)
        sl_hi = [slice(None)] * z.ndim
        sl_lo = [slice(None)] * z.ndim
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(None, -1)
        d[tuple(sl_lo)] = z[tuple(sl_hi)] - z[tuple(sl_lo)]
        out.append(d)
    return np.stack(out)


def _DT_from_oracle(orc, p):
    """D^T p read off the prox with no inner iterations: z = v - tau D^T p (v = 0, tau = 1)."""
    shape = p.shape[1:]
    z = orc.tv_prox_fgp(np.zeros(shape), 1.0, 0, nonneg=False, dual=p.copy())
    return -z


@pytest.mark.parametrize("shape", [(9, 13), (5, 7, 6)])
def test_divergence_is_adjoint_of_gradient(orc, shape):
    rng = np.random.default_rng(0)
    z = rng.standard_normal(shape)
    d = len(shape)
    p = rng.standard_normal((d,) + ((1,) if d == 2 else ()) + shape)
    Dz = _D(z)
    DTp = _DT_from_oracle(orc, p).reshape(shape)
    lhs = np.sum(Dz * p.reshape((d,) + shape))
    rhs = np.sum(z * DTp)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_tv_values(orc):
    ny, nx, a, b = 6, 10, 0.25, 1.75
    v = np.full((ny, nx), a)
    v[:, nx // 2:] = b
    assert orc.tv(v) == ny * (b - a)
    rng = np.random.default_rng(1)
    z = rng.standard_normal((7, 8))
    assert abs(orc.tv(z) - np.sum(np.sqrt(np.sum(_D(z) ** 2, axis=0)))) <= 1e-12 * orc.tv(z)
    z3 = rng.standard_normal((3, 4, 5))
    assert abs(orc.tv(z3) - np.sum(np.sqrt(np.sum(_D(z3) ** 2, axis=0)))) <= 1e-12 * orc.tv(z3)


def test_constant_image_is_fixed(orc):
    v = np.full((12, 15), 0.7)
    for nonneg in (False, True):
        z = orc.tv_prox_fgp(v, 0.3, 50, nonneg=nonneg)
        assert np.array_equal(z, v)


def test_tau_zero_is_identity_or_projection(orc):
    rng = np.random.default_rng(2)
    v = rng.standard_normal((6, 9))
    dual = rng.standard_normal((2, 1, 6, 9))
    d0 = dual.copy()
    assert np.array_equal(orc.tv_prox_fgp(v, 0.0, 10, nonneg=False, dual=dual), v)
    assert np.array_equal(orc.tv_prox_fgp(v, 0.0, 10, nonneg=True, dual=dual), np.maximum(v, 0.0))
    assert np.array_equal(dual, d0)   # dual untouched when tau = 0


@pytest.mark.parametrize("a,b,tau", [(0.3, 1.1, 0.5), (0.2, 0.4, 1.5)])
def test_two_level_closed_form(orc, a, b, tau):
    # A vertical step reduces to 1D TV denoising: each half moves towards the other by
    # tau / (nx/2) while the jump stays non-negative, else both meet at the mean.
    ny, nx = 6, 16
    v = np.full((ny, nx), a)
    v[:, nx // 2:] = b
    shift = 2.0 * tau / nx
    ref = v.copy()
    if b - a >= 2 * shift:
        ref[:, : nx // 2] += shift
        ref[:, nx // 2:] -= shift
    else:
        ref[:] = (a + b) / 2
    z = orc.tv_prox_fgp(v, tau, 20000, nonneg=True)
    assert np.max(np.abs(z - ref)) <= 1e-10


def test_brute_force_8x8_duality_gap(orc):
    # Unconstrained prox: primal 1/2||z-v||^2 + tau TV(z) and dual 1/2||v||^2 - 1/2||v - tau D^T p||^2
    # meet at the optimum, with z = v - tau D^T p and |p_ij| <= 1.
    rng = np.random.default_rng(3)
    v = rng.uniform(0.0, 1.0, (8, 8))
    tau = 0.1
    dual = np.zeros((2, 1, 8, 8))
    z = orc.tv_prox_fgp(v, tau, 20000, nonneg=False, dual=dual)
    DTp = _DT_from_oracle(orc, dual).reshape(8, 8)
    assert np.max(np.sqrt(np.sum(dual ** 2, axis=0))) <= 1.0 + 1e-15
    primal = 0.5 * np.sum((z - v) ** 2) + tau * orc.tv(z)
    dualv = 0.5 * np.sum(v ** 2) - 0.5 * np.sum((v - tau * DTp) ** 2)
    assert primal - dualv <= 1e-12
    assert primal - dualv >= -1e-12
    assert np.max(np.abs(z - (v - tau * DTp))) <= 1e-15


@pytest.mark.slow
@pytest.mark.parametrize("nonneg", [False, True])
def test_brute_force_8x8_vs_independent_solver(orc, nonneg):
    rng = np.random.default_rng(4)
    v = rng.standard_normal((8, 8)) * 0.5 + (0.0 if nonneg else 0.5)
    tau = 0.1
    z = orc.tv_prox_fgp(v, tau, 20000, nonneg=nonneg)
    zd = orc.tv_prox_dpg(v, tau, 1000000, nonneg=nonneg)
    assert np.max(np.abs(z - zd)) <= 1e-9
    if nonneg:
        assert np.all(z >= 0.0) and np.any(z == 0.0)


def test_brute_force_3d_duality_gap(orc):
    # A volume that varies along z: the unconstrained 3D prox closes the primal-dual gap,
    # primal 1/2||z - v||^2 + tau TV3(z) (TV3 from the differences written in this file) against
    # dual 1/2||v||^2 - 1/2||v - tau D^T p|| ^2, with z = v - tau D^T p and |p_ijk| <= 1.
    rng = np.random.default_rng(8)
    v = rng.uniform(0.0, 1.0, (3, 5, 6))
    tau = 0.1
    dual = np.zeros((3, 3, 5, 6))
    z = orc.tv_prox_fgp(v, tau, 40000, nonneg=False, dual=dual)
    DTp = _DT_from_oracle(orc, dual).reshape(v.shape)
    tv3 = float(np.sum(np.sqrt(np.sum(_D(z) ** 2, axis=0))))
    assert np.max(np.sqrt(np.sum(dual ** 2, axis=0))) <= 1.0 + 1e-15
    primal = 0.5 * np.sum((z - v) ** 2) + tau * tv3
    dualv = 0.5 * np.sum(v ** 2) - 0.5 * np.sum((v - tau * DTp) ** 2)
    assert abs(primal - dualv) <= 1e-10, primal - dualv
    assert np.max(np.abs(z - (v - tau * DTp))) <= 1e-15
    # the z coupling matters: the slice-wise 2D prox is not the answer
    z2 = np.stack([orc.tv_prox_fgp(v[k], tau, 20000, nonneg=False) for k in range(3)])
    assert np.max(np.abs(z - z2)) >= 1e-3


def test_3d_constant_along_z_matches_2d(orc):
    # The z differences of a z-constant volume are zero, so the 3D prox is the 2D prox of each
    # slice (at convergence; the 3D step size 1/(12 tau) differs from the 2D 1/(8 tau)).
    rng = np.random.default_rng(5)
    sl = rng.uniform(0.0, 1.0, (7, 9))
    vol = np.repeat(sl[None], 4, axis=0)
    tau = 0.08
    z2 = orc.tv_prox_fgp(sl, tau, 20000, nonneg=True)
    z3 = orc.tv_prox_fgp(vol, tau, 20000, nonneg=True)
    for k in range(4):
        assert np.max(np.abs(z3[k] - z2)) <= 1e-9


def test_warm_start_is_a_continuation(orc):
    # Two warm-started calls of K iterations reach the same point as a restart-free run would
    # approach: the dual carries the state, so 2 x 1000 iterations land close to the optimum.
    rng = np.random.default_rng(6)
    v = rng.uniform(0.0, 1.0, (10, 10))
    tau = 0.05
    ref = orc.tv_prox_fgp(v, tau, 50000, nonneg=True)
    dual = np.zeros((2, 1, 10, 10))
    z = None
    for _ in range(20):
        z = orc.tv_prox_fgp(v, tau, 10, nonneg=True, dual=dual)
    cold = orc.tv_prox_fgp(v, tau, 10, nonneg=True)
    assert np.max(np.abs(z - ref)) < np.max(np.abs(cold - ref))
