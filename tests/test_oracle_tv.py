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


# ---------------------------------------------------------------------------------------------
# FGP at a finite number of inner iterations, derived by hand (Beck & Teboulle 2009, cited in
# Sec. 2.1 for the TV prox).  The solver runs a fixed, small number of inner iterations, so the
# trajectory itself (step 1/(4 d tau), t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, momentum
# (t_k - 1) / t_{k+1} first felt at the third iteration, output from p_K rather than the
# extrapolated r) is what the GPU is compared with; these cases fix it independently.
# ---------------------------------------------------------------------------------------------

def _t_sequence(k):
    t = [None, 1.0]                       # t_1 = 1
    for _ in range(k):
        t.append((1.0 + np.sqrt(1.0 + 4.0 * t[-1] ** 2)) / 2.0)
    return t


def _scalar_fgp_duals(step_map, K):
    """p_1 .. p_K of a prox whose dual reduces to one scalar q: the ascent step q+ = step_map(r)
    followed by the projection onto [-1, 1] (the unit ball of a pixel with one non-zero
    component), r_1 = 0, r_{k+1} = p_k + ((t_k - 1) / t_{k+1}) (p_k - p_{k-1})."""
    t = _t_sequence(K + 1)
    p_prev, r, out = 0.0, 0.0, []
    for k in range(1, K + 1):
        p = min(max(step_map(r), -1.0), 1.0)
        r = p + ((t[k] - 1.0) / t[k + 1]) * (p - p_prev)
        p_prev = p
        out.append(p)
    return out


def test_fgp_two_pixels_by_hand(orc):
    # 1 x 2 image v = (0, 1), tau = 1/2, no constraint.  Only the x-difference of pixel 0 is
    # non-zero, so the dual is one scalar q:  z = (tau q, 1 - tau q),  Dz = 1 - 2 tau q = 1 - q,
    # and the ascent step 1/(8 tau) = 1/4 gives q+ = r + (1 - r)/4 = (3 r + 1)/4.
    #   K = 1: r_1 = 0         -> p_1 = 1/4
    #   K = 2: r_2 = p_1       -> p_2 = 7/16          (beta_1 = (t_1 - 1)/t_2 = 0)
    #   K = 3: r_3 = p_2 + beta_2 (p_2 - p_1) = 7/16 + (3/16) beta_2,  beta_2 = (t_2 - 1)/t_3
    #   K = 4: r_4 = p_3 + beta_3 (p_3 - p_2)
    # and z_K = (p_K / 2, 1 - p_K / 2).
    t = _t_sequence(4)
    beta2 = (t[2] - 1.0) / t[3]
    beta3 = (t[3] - 1.0) / t[4]
    p1 = 0.25
    p2 = 7.0 / 16.0
    p3 = (3.0 * (7.0 / 16.0 + (3.0 / 16.0) * beta2) + 1.0) / 4.0
    p4 = (3.0 * (p3 + beta3 * (p3 - p2)) + 1.0) / 4.0
    assert abs(t[2] - (1.0 + np.sqrt(5.0)) / 2.0) < 1e-15
    v = np.array([[0.0, 1.0]])
    for K, pk in zip((1, 2, 3, 4), (p1, p2, p3, p4)):
        dual = np.zeros((2, 1, 1, 2))
        z = orc.tv_prox_fgp(v, 0.5, K, nonneg=False, dual=dual)
        assert np.allclose(z.ravel(), [pk / 2.0, 1.0 - pk / 2.0], rtol=0, atol=1e-15), K
        want = np.zeros((2, 1, 1, 2))
        want[0, 0, 0, 0] = pk
        assert np.allclose(dual, want, rtol=0, atol=1e-15), K
    # the recursion written as a loop agrees with the unrolled values above
    assert np.allclose(_scalar_fgp_duals(lambda r: (3.0 * r + 1.0) / 4.0, 4),
                       [p1, p2, p3, p4], rtol=0, atol=1e-16)


def test_fgp_rows_slices_and_constraint_by_hand(orc):
    # The same two-pixel step along y (2 x 1 image): the dual sits in the y component.
    K = 5
    qs = _scalar_fgp_duals(lambda r: (3.0 * r + 1.0) / 4.0, K)
    dual = np.zeros((2, 1, 2, 1))
    z = orc.tv_prox_fgp(np.array([[0.0], [1.0]]), 0.5, K, nonneg=False, dual=dual)
    assert np.allclose(z.ravel(), [qs[-1] / 2.0, 1.0 - qs[-1] / 2.0], rtol=0, atol=1e-15)
    assert abs(dual[1, 0, 0, 0] - qs[-1]) <= 1e-15 and np.count_nonzero(dual) == 1
    # Along z (1 x 1 x 2 volume, 3D TV): step 1/(12 tau), so with tau = 1/2
    # q+ = r + (1 - r)/6 = (5 r + 1)/6:  p_1 = 1/6, p_2 = 11/36, ...
    qs3 = _scalar_fgp_duals(lambda r: (5.0 * r + 1.0) / 6.0, K)
    assert abs(qs3[0] - 1.0 / 6.0) < 1e-16 and abs(qs3[1] - 11.0 / 36.0) < 1e-16
    dual = np.zeros((3, 2, 1, 1))
    z = orc.tv_prox_fgp(np.array([[[0.0]], [[1.0]]]), 0.5, K, nonneg=False, dual=dual)
    assert np.allclose(z.ravel(), [qs3[-1] / 2.0, 1.0 - qs3[-1] / 2.0], rtol=0, atol=1e-15)
    assert abs(dual[2, 0, 0, 0] - qs3[-1]) <= 1e-15 and np.count_nonzero(dual) == 1
    # With the constraint: v = (-1, 1), tau = 1/2.  z = P_C(-1 + q/2, 1 - q/2) = (0, 1 - q/2)
    # while q < 2, so Dz = 1 - q/2 and q+ = r + (1 - r/2)/4 = 7r/8 + 1/4:  p_1 = 1/4,
    # p_2 = 15/32, p_3 = 7/8 (15/32 + (7/32) beta_2) + 1/4.  The momentum carries p_5 past 1,
    # where the ball projection clips it: z_5 = (0, 1/2), the exact prox (z_0 = 0 and
    # 1/2 (z_1 - 1)^2 + z_1 / 2 minimal at 1/2).
    t = _t_sequence(3)
    qc = _scalar_fgp_duals(lambda r: 7.0 * r / 8.0 + 0.25, K)
    assert abs(qc[1] - 15.0 / 32.0) < 1e-16
    assert abs(qc[2] - (7.0 / 8.0 * (15.0 / 32.0 + 7.0 / 32.0 * (t[2] - 1.0) / t[3]) + 0.25)) < 1e-15
    assert qc[3] < 1.0 and qc[4] == 1.0
    for k in (3, 5):
        dual = np.zeros((2, 1, 1, 2))
        z = orc.tv_prox_fgp(np.array([[-1.0, 1.0]]), 0.5, k, nonneg=True, dual=dual)
        assert np.allclose(z.ravel(), [0.0, 1.0 - qc[k - 1] / 2.0], rtol=0, atol=1e-15), k
        assert abs(dual[0, 0, 0, 0] - qc[k - 1]) <= 1e-15, k


def test_fgp_isotropic_ball_projection_by_hand(orc):
    # 2 x 2 image v = [[0, 1], [1, 1]], tau = 1/5, step 1/(8 tau) = 5/8.
    # K = 1: Dz at (0,0) = (1, 1), zero elsewhere, so p_1(0,0) = (5/8, 5/8) (norm < 1) and
    #        z = v - tau D^T p_1 with (D^T p_1) = [[-5/4, 5/8], [5/8, 0]]:
    #        z_1 = [[1/4, 7/8], [7/8, 1]].
    # K = 2: r_2 = p_1.  D z_1: (0,0) -> (5/8, 5/8); x-difference at (1,0) -> 1/8;
    #        y-difference at (0,1) -> 1/8.  Before projection p(0,0) = (65/64, 65/64), whose
    #        norm 65 sqrt(2)/64 > 1, so the isotropic projection gives (1/sqrt 2, 1/sqrt 2)
    #        (clipping each component, the anisotropic rule, would give (1, 1)); p(1,0) has
    #        x = 5/64 and p(0,1) has y = 5/64.  Then
    #        D^T p_2 = [[-sqrt 2, 1/sqrt 2 - 5/64], [1/sqrt 2 - 5/64, 5/32]].
    v = np.array([[0.0, 1.0], [1.0, 1.0]])
    tau = 0.2
    dual = np.zeros((2, 1, 2, 2))
    z1 = orc.tv_prox_fgp(v, tau, 1, nonneg=False, dual=dual)
    assert np.allclose(z1.reshape(2, 2), [[0.25, 0.875], [0.875, 1.0]], rtol=0, atol=1e-15)
    assert np.allclose(dual[:, 0, 0, 0], [0.625, 0.625], rtol=0, atol=1e-15)
    s = 1.0 / np.sqrt(2.0)
    dual = np.zeros((2, 1, 2, 2))
    z2 = orc.tv_prox_fgp(v, tau, 2, nonneg=False, dual=dual)
    dtp = np.array([[-np.sqrt(2.0), s - 5.0 / 64.0], [s - 5.0 / 64.0, 5.0 / 32.0]])
    assert np.allclose(z2.reshape(2, 2), v - tau * dtp, rtol=0, atol=1e-15)
    want = np.zeros((2, 2, 2))
    want[0, 0, 0] = want[1, 0, 0] = s          # pixel (0,0): x and y components
    want[1, 0, 1] = 5.0 / 64.0                 # y-difference of pixel (0,1)
    want[0, 1, 0] = 5.0 / 64.0                 # x-difference of pixel (1,0)
    assert np.allclose(dual[:, 0], want, rtol=0, atol=1e-15)


def test_fgp_dual_gap_obeys_the_fista_rate(orc):
    # FGP is FISTA on the dual  min_{|p_pixel| <= 1} q(p) = 1/2 ||v - tau D^T p||^2, whose
    # gradient is tau^2 ||D||^2 <= 8 tau^2 Lipschitz; Beck & Teboulle's bound for it reads
    # q(p_k) - q* <= 2 (8 tau^2) ||p_0 - p*||^2 / (k + 1)^2 for every k and every minimiser p*.
    rng = np.random.default_rng(12)
    v = rng.standard_normal((8, 8))
    tau = 0.3
    pstar = np.zeros((2, 1, 8, 8))
    zstar = orc.tv_prox_dpg(v, tau, 200_000, nonneg=False, dual=pstar)
    qstar = 0.5 * np.sum(zstar ** 2)
    bound_c = 2.0 * 8.0 * tau ** 2 * np.sum(pstar ** 2)
    for k in (1, 2, 3, 5, 10, 20, 50, 100, 200):
        zk = orc.tv_prox_fgp(v, tau, k, nonneg=False, dual=np.zeros((2, 1, 8, 8)))
        gap = 0.5 * np.sum(zk ** 2) - qstar
        assert gap >= -1e-12
        assert gap <= bound_c / (k + 1) ** 2 + 1e-12, k
