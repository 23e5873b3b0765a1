"""Pins of the oracle's reference solver x* (Sec. 2.1: a separate primal-dual method; the
data-splitting figure: PDHG with diagonal preconditioning, Chambolle & Pock 2011) (no GPU).

x* is pinned by what characterises the minimiser of Eq. 5: with alpha = 0 and no constraint it
is the least-squares solution; otherwise the optimality conditions hold at the limit (the dual
y1 equals the residual Ax - b, A^T y1 + D^T y2 vanishes on the support of x and is >= 0 where
x = 0, y2 lies in the alpha-ball and equals alpha Dx/|Dx| where Dx != 0); and an independent
method, FISTA (pinned on its own), reaches the same point.
"""
import numpy as np


def _D(x):
    # forward differences with a zero last difference, components (x, y)
    p = np.zeros((2,) + x.shape)
    p[0][..., :-1] = x[..., 1:] - x[..., :-1]
    p[1][:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    return p


def _DT(p):
    # the adjoint: <D x, p> = <x, D^T p>
    out = np.zeros(p.shape[1:])
    out[..., 1:] += p[0][..., :-1]
    out[..., :-1] -= p[0][..., :-1]
    out[:, 1:, :] += p[1][:, :-1, :]
    out[:, :-1, :] -= p[1][:, :-1, :]
    return out


def test_difference_operator_adjoint():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 7, 9))
    p = rng.standard_normal((2, 1, 7, 9))
    assert abs(np.sum(_D(x) * p) - np.sum(x * _DT(p))) <= 1e-12 * np.sum(np.abs(x))


def test_pdhg_least_squares_limit(orc):
    g = orc.Geometry(5, 5, n_angles=20, n_bins=9, n_subsets=1)
    M = np.zeros((180, 25))
    for e in range(25):
        v = np.zeros(25)
        v[e] = 1.0
        M[:, e] = orc.project(g, v.reshape(1, 5, 5)).ravel()
    b = np.random.default_rng(2).standard_normal((1, 20, 9))
    xstar = np.linalg.lstsq(M, b.ravel(), rcond=None)[0]
    x, y1, _ = orc.pdhg(g, b, alpha=0.0, n_iters=5000, nonneg=False)
    assert np.linalg.norm(x.ravel() - xstar) <= 1e-12 * np.linalg.norm(xstar)
    r = (M @ xstar - b.ravel())
    assert np.linalg.norm(y1.ravel() - r) <= 1e-10 * np.linalg.norm(r)


def test_pdhg_optimality_conditions(orc):
    g = orc.Geometry(12, 12, n_angles=24, n_bins=18, n_subsets=1)
    b = np.abs(np.random.default_rng(0).standard_normal((1, 24, 18))) * 5.0
    alpha = 2.0
    x, y1, y2 = orc.pdhg(g, b, alpha=alpha, n_iters=10000, nonneg=True)
    r = orc.project(g, x) - b
    assert np.linalg.norm(y1 - r) <= 1e-12 * np.linalg.norm(r)
    grad = orc.backproject(g, y1) + _DT(y2)
    scale = np.max(np.abs(orc.backproject(g, r)))
    on = x > 1e-8
    assert 0 < on.sum() < x.size                       # the constraint is active somewhere
    assert np.max(np.abs(grad[on])) <= 1e-12 * scale
    assert grad[~on].min() >= -1e-12 * scale
    nrm = np.sqrt(np.sum(y2 ** 2, axis=0))
    assert nrm.max() <= alpha * (1 + 1e-12)
    dx = _D(x)
    ndx = np.sqrt(np.sum(dx ** 2, axis=0))
    edge = ndx > 1e-6
    assert np.max(np.abs(y2[:, edge] - alpha * dx[:, edge] / ndx[edge])) <= 1e-9 * alpha


def test_pdhg_agrees_with_fista(orc):
    g = orc.Geometry(12, 12, n_angles=24, n_bins=18, n_subsets=1)
    b = np.abs(np.random.default_rng(0).standard_normal((1, 24, 18))) * 5.0
    x, _, _ = orc.pdhg(g, b, alpha=2.0, n_iters=10000, nonneg=True)
    xf, _, _ = orc.fista(g, b, gamma=1.0 / orc.lipschitz(g, 300), alpha=2.0, fgp_inner=200,
                         n_iters=3000, nonneg=True)
    assert np.linalg.norm(xf - x) <= 1e-10 * np.linalg.norm(x)
