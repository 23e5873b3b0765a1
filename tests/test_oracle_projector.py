"""Pins of the oracle's projector, adjoint, gradients and Lipschitz constant (no GPU).

Each test checks the FP64 oracle against something other than itself: a closed form, a
hand derivation, a textbook routine, or an invariant the mathematics fixes.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2602_09527_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------------------------
# Closed forms of the forward projector (Sec. 2.1: A is the discrete Radon transform).
# ---------------------------------------------------------------------------------------------

def test_theta0_is_column_sums_bitwise(orc):
    # theta = 0, B - nx even: every sample lands on a pixel centre (w = 0), so each bin is the
    # plain column sum of the matching column, accumulated top to bottom.
    nx, ny, B = 12, 9, 16
    g = orc.Geometry(nx, ny, n_angles=4, n_bins=B)
    x = _rng(1).standard_normal((1, ny, nx))
    y = orc.project(g, x)[0, 0]
    shift = (B - nx) // 2
    for u in range(B):
        j = u - shift
        ref = 0.0
        if 0 <= j < nx:
            for i in range(ny):
                ref += x[0, i, j]
        assert y[u] == ref


def test_theta_half_pi_is_row_sums(orc):
    # theta = pi/2 is walked column by column and gives the row sums.
    nx, ny, B = 10, 14, 18
    g = orc.Geometry(nx, ny, n_angles=2, n_bins=B)
    x = _rng(2).standard_normal((1, ny, nx))
    y = orc.project(g, x)[0, 1]
    shift = (B - ny) // 2
    ref = np.zeros(B)
    for u in range(B):
        i = u - shift
        if 0 <= i < ny:
            ref[u] = x[0, i, :].sum()
    assert np.max(np.abs(y - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_constant_image_theta0(orc):
    nx, ny, B = 16, 11, 20
    g = orc.Geometry(nx, ny, n_angles=3, n_bins=B)
    y = orc.project(g, np.ones((1, ny, nx)))[0, 0]
    shift = (B - nx) // 2
    expect = np.array([ny if 0 <= u - shift < nx else 0.0 for u in range(B)], dtype=float)
    assert np.array_equal(y, expect)


def test_hand_derived_3x3(orc):
    spec = json.load(open(os.path.join(GOLDEN, "joseph_3x3.json")))
    r5 = math.sqrt(5.0)
    W = np.zeros((3, 9))
    for u, i, j, expr in spec["weights_atan_half"]["entries"]:
        W[u, 3 * i + j] = eval(expr, {"r5": r5})
    # the mirror angle has the same weights with i and j swapped
    Wt = np.zeros((3, 9))
    for u, i, j, expr in spec["weights_atan_half"]["entries"]:
        Wt[u, 3 * j + i] = eval(expr, {"r5": r5})
    g = orc.Geometry(3, 3, n_angles=2, n_bins=3, angles=np.array([math.atan(0.5), math.atan(2.0)]))
    M = np.zeros((2, 3, 9))
    for e in range(9):
        v = np.zeros(9)
        v[e] = 1.0
        M[:, :, e] = orc.project(g, v.reshape(1, 3, 3))[0]
    assert np.max(np.abs(M[0] - W)) < 1e-14
    assert np.max(np.abs(M[1] - Wt)) < 1e-14


def _gauss_errors(orc, sigma, n=128, A=16):
    x0, y0 = 3.3, -5.1
    xs = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(xs, xs)
    img = np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * sigma ** 2))
    g = orc.Geometry(n, n, n_angles=A, n_bins=n)
    y = orc.project(g, img[None])[0]
    th = np.arange(A) * np.pi / A
    s = np.arange(n) - (n - 1) / 2.0
    s0 = x0 * np.cos(th)[:, None] + y0 * np.sin(th)[:, None]
    ref = math.sqrt(2 * math.pi) * sigma * np.exp(-(s[None, :] - s0) ** 2 / (2 * sigma ** 2))
    return np.max(np.abs(y - ref)) / np.max(ref)


def test_gaussian_blob_closed_form(orc):
    # A Gaussian projects to a Gaussian: sqrt(2 pi) sigma exp(-(s-s0)^2 / 2 sigma^2).  Linear
    # interpolation is second order, so halving sigma roughly quadruples the error.
    e8 = _gauss_errors(orc, 8.0)
    e4 = _gauss_errors(orc, 4.0)
    assert e8 <= 5e-3
    assert 2.5 <= e4 / e8 <= 6.0


def _disc_error(orc, r, n):
    ells = [synth.Ellipse(0.0, 0.0, r / (n / 2), r / (n / 2), 0.0, 1.0)]
    img = synth.rasterize(ells, n, n, supersample=8)
    A = 12
    g = orc.Geometry(n, n, n_angles=A, n_bins=n)
    y = orc.project(g, img)[0]
    s = np.arange(n) - (n - 1) / 2.0
    chord = 2.0 * np.sqrt(np.maximum(r * r - s * s, 0.0))
    return np.mean(np.abs(y - chord[None, :])) / (2 * r)


def test_disc_chord(orc):
    # A disc of radius r projects to the chord 2 sqrt(r^2 - s^2) at every angle; the pixelised
    # edge makes the error first order in the pixel size.
    e40 = _disc_error(orc, 40.0, 128)
    e20 = _disc_error(orc, 20.0, 64)
    assert e40 <= 1e-2
    assert 1.4 <= e20 / e40 <= 2.8


def test_ellipse_closed_form(orc):
    # Random ellipses: the projection approaches the exact line integrals (Kak & Slaney); the
    # pixelised edges make the error first order, so doubling the resolution halves it.
    ells = synth.random_ellipses(7, 10)
    errs = []
    for n in (64, 128):
        A = 30
        img = synth.rasterize(ells, n, n, supersample=4)
        exact = synth.analytic_sinogram(ells, n, n, A, n)
        g = orc.Geometry(n, n, n_angles=A, n_bins=n)
        y = orc.project(g, img)
        errs.append(np.linalg.norm(y - exact) / np.linalg.norm(exact))
    assert errs[1] <= 1.5e-2
    assert 1.6 <= errs[0] / errs[1] <= 2.5


# ---------------------------------------------------------------------------------------------
# Adjoint, subsets, gradients.
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(16, 16, 24, 24, 4), (13, 9, 31, 17, 5), (20, 12, 7, 29, 7)])
def test_dot_test(orc, shape):
    nx, ny, A, B, N = shape
    g = orc.Geometry(nx, ny, n_angles=A, n_bins=B, n_subsets=N, nz=2, off=0.37)
    rng = _rng(3)
    for subset in [-1] + list(range(N)):
        na = g.subset_size(subset)
        x = rng.standard_normal((2, ny, nx))
        y = rng.standard_normal((2, na, B))
        lhs = float(np.sum(orc.project(g, x, subset) * y))
        rhs = float(np.sum(x * orc.backproject(g, y, subset)))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_subsets_stack_to_full(orc):
    nx, ny, A, B, N = 14, 14, 23, 20, 5   # A not divisible by N: ragged subsets
    g = orc.Geometry(nx, ny, n_angles=A, n_bins=B, n_subsets=N)
    x = _rng(4).standard_normal((1, ny, nx))
    full = orc.project(g, x, -1)
    sizes = [g.subset_size(i) for i in range(N)]
    assert sum(sizes) == A and max(sizes) - min(sizes) <= 1
    for i in range(N):
        yi = orc.project(g, x, i)
        assert np.array_equal(yi[0], full[0, i::N])
    # sum_i A_i^T A_i v = A^T A v
    v = _rng(5).standard_normal((1, ny, nx))
    acc = sum(orc.backproject(g, orc.project(g, v, i), i) for i in range(N))
    ref = orc.backproject(g, orc.project(g, v, -1), -1)
    assert np.max(np.abs(acc - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_single_rays_and_pixels(orc):
    nx, ny, A, B, N = 17, 11, 13, 21, 3
    g = orc.Geometry(nx, ny, n_angles=A, n_bins=B, n_subsets=N, nz=2, du=0.8, off=-0.6)
    rng = _rng(6)
    x = rng.standard_normal((2, ny, nx))
    full = orc.project(g, x)
    zs, ks, us = rng.integers(0, 2, 50), rng.integers(0, A, 50), rng.integers(0, B, 50)
    assert np.array_equal(orc.project_rays(g, x, zs, ks, us), full[zs, ks, us])
    for subset in (-1, 1):
        y = rng.standard_normal((2, g.subset_size(subset), B))
        bp = orc.backproject(g, y, subset)
        zi, ii, jj = rng.integers(0, 2, 40), rng.integers(0, ny, 40), rng.integers(0, nx, 40)
        got = orc.backproject_pixels(g, y, zi, ii, jj, subset)
        assert np.max(np.abs(got - bp[zi, ii, jj])) <= 1e-13 * np.max(np.abs(bp))


def test_gradients(orc):
    nx, ny, A, B, N = 16, 12, 20, 22, 4
    g = orc.Geometry(nx, ny, n_angles=A, n_bins=B, n_subsets=N)
    rng = _rng(7)
    x = rng.standard_normal((1, ny, nx))
    b = rng.standard_normal((1, A, B))
    # sum of subset gradients = A^T (A x - b): checks the gather of b_i from b
    gf = orc.grad_full(g, x, b)
    ref = orc.backproject(g, orc.project(g, x) - b)
    assert np.max(np.abs(gf - ref)) <= 1e-12 * np.max(np.abs(ref))
    # f is quadratic, so a central difference is exact up to rounding
    for _ in range(3):
        v = rng.standard_normal(x.shape)
        eps = 1e-3
        fd = (orc.data_fit(g, x + eps * v, b) - orc.data_fit(g, x - eps * v, b)) / (2 * eps)
        assert abs(fd - np.sum(gf * v)) <= 1e-8 * max(1.0, abs(fd))
    # SVRG estimator: (1/N) sum_i [N (grad_i(x) - grad_i(xs)) + grad(xs)] = grad f(x)
    xs = rng.standard_normal(x.shape)
    gs = orc.grad_full(g, xs, b)
    est = sum(N * (orc.grad_subset(g, x, b, i) - orc.grad_subset(g, xs, b, i)) + gs
              for i in range(N)) / N
    assert np.max(np.abs(est - gf)) <= 1e-12 * np.max(np.abs(gf))
    # at x = xs the estimator is exactly the snapshot gradient
    for i in range(N):
        gi = orc.grad_subset(g, xs, b, i)
        assert np.array_equal(N * (gi - gi) + gs, gs)


def test_lipschitz_vs_dense_eigensolver(orc):
    g = orc.Geometry(16, 16, n_angles=24, n_bins=24, n_subsets=3)
    L = orc.lipschitz(g, 500)
    M = np.zeros((24 * 24, 256))
    for e in range(256):
        v = np.zeros(256)
        v[e] = 1.0
        M[:, e] = orc.project(g, v.reshape(1, 16, 16)).ravel()
    lam = np.linalg.eigvalsh(M.T @ M)[-1]
    assert abs(L - lam) <= 1e-10 * lam
