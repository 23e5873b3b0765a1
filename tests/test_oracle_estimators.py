"""Pins of the oracle's other estimators of the table beside Algorithm 1 (loopless SVRG, SAGA)
and of FISTA (no GPU).

The paper prints no iterates for these either, so each part is pinned by what the definitions
and the mathematics fix: the general loop with the SVRG estimator is the already pinned SVRG
loop; loopless SVRG refreshed exactly at epoch starts is SVRG; with one subset every estimator
is the full gradient; the SAGA table keeps vbar = sum_i v_i and v_i = grad f_i at the last
visit; with a trivial prox and p = 1 the stochastic methods converge to the least-squares
solution; the first FISTA step is the ISTA step, and FISTA meets the O(1/k^2) bound of Beck and
Teboulle (2009, Theorem 4.4).
"""
import numpy as np
import pytest


def _problem(orc, nx=12, ny=12, A=24, B=18, N=4, seed=0):
    g = orc.Geometry(nx, ny, n_angles=A, n_bins=B, n_subsets=N)
    rng = np.random.default_rng(seed)
    b = np.abs(rng.standard_normal((1, A, B))) * 5.0
    return g, b


def _matrix(orc, g):
    n = g.nx * g.ny
    M = np.zeros((g.n_angles * g.n_bins, n))
    for e in range(n):
        v = np.zeros(n)
        v[e] = 1.0
        M[:, e] = orc.project(g, v.reshape(1, g.ny, g.nx)).ravel()
    return M


# ---------------------------------------------------------------------------------------------
# Refresh stream of the loopless SVRG estimator.
# ---------------------------------------------------------------------------------------------

def test_refresh_coins_definition_and_statistics(orc):
    seed = 31
    rho = orc.refresh_coins(seed, 0, 64, 7)
    for k in range(64):
        u = orc.splitmix64(seed, (1 << 62) + k)
        assert rho[k] == int((u >> 11) < (1 << 53) // 7)
    n = 1_000_000
    for N in (3, 10, 30):
        r = orc.refresh_coins(12345, 0, n, N)
        q = 1.0 / N
        assert abs(int(r.sum()) - n * q) <= 5 * np.sqrt(n * q * (1 - q))
    assert orc.refresh_coins(3, 0, 1000, 1).all()
    tail = orc.refresh_coins(5, 140, 160, 9)
    assert np.array_equal(orc.refresh_coins(5, 0, 300, 9)[140:], tail)


# ---------------------------------------------------------------------------------------------
# The general loop against the pinned SVRG loop, and loopless SVRG.
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("k0,tol", [(0, 0.0), (8, 0.0), (0, 0.3)])
def test_svrg_estimator_matches_svrg_loop(orc, k0, tol):
    g, b = _problem(orc, seed=1)
    gamma = 1.0 / orc.lipschitz(g, 300)
    kw = dict(gamma=gamma, p=0.3, alpha=1.2, fgp_inner=12, nonneg=True, seed=17, k0=k0, tol=tol)
    a = orc.proxskip_svrg(g, b, n_epochs=5, **kw)
    c = orc.proxskip(g, b, estimator="svrg", n_epochs=5, **kw)
    for u, v in zip(a[:3], c[:3]):
        assert np.array_equal(u, v)
    assert a[3] == c[3]
    assert np.array_equal(a[4], c[4])


def test_lsvrg_refreshed_at_epoch_starts_is_svrg(orc):
    g, b = _problem(orc, seed=2)
    N = g.n_subsets
    gamma = 1.0 / orc.lipschitz(g, 300)
    K = 6 * N
    refresh = (np.arange(K) % N == 0).astype(np.uint8)
    kw = dict(gamma=gamma, p=0.25, alpha=0.8, fgp_inner=10, nonneg=True, seed=4, n_iters=K)
    s = orc.proxskip(g, b, estimator="svrg", **kw)
    ls = orc.proxskip(g, b, estimator="lsvrg", refresh=refresh, **kw)
    for u, v in zip(s[:3], ls[:3]):
        assert np.array_equal(u, v)


def test_lsvrg_snapshot_bookkeeping(orc):
    # prox = identity (alpha = 0, no constraint), p = 1: x+ = x - gamma G.  A refresh makes
    # G = grad f(x); without one, G keeps the last snapshot.
    g, b = _problem(orc, seed=3)
    N = g.n_subsets
    gamma = 0.5 / orc.lipschitz(g, 300)
    rng = np.random.default_rng(0)
    x0 = rng.random((1, g.ny, g.nx))
    sub = np.array([2, 0, 3], dtype=np.int32)
    refresh = np.array([1, 0, 1], dtype=np.uint8)
    x = orc.proxskip(g, b, estimator="lsvrg", gamma=gamma, p=1.0, alpha=0.0, fgp_inner=0,
                     nonneg=False, plain=True, n_iters=3, sub=sub, refresh=refresh, x=x0)[0]
    x1 = x0 - gamma * orc.grad_full(g, x0, b)
    G1 = N * (orc.grad_subset(g, x1, b, 0) - orc.grad_subset(g, x0, b, 0)) + orc.grad_full(g, x0, b)
    x2 = x1 - gamma * G1
    x3 = x2 - gamma * orc.grad_full(g, x2, b)
    assert np.max(np.abs(x - x3)) <= 1e-13 * np.max(np.abs(x3))


def test_single_subset_estimators_are_the_full_gradient(orc):
    # N = 1: every estimator is grad f(x_k), so all three give deterministic ProxSkip.
    g, b = _problem(orc, N=1, seed=6)
    gamma = 1.0 / orc.lipschitz(g, 300)
    kw = dict(gamma=gamma, p=0.4, alpha=1.5, fgp_inner=15, nonneg=True, seed=8, n_epochs=20)
    s = orc.proxskip(g, b, estimator="svrg", **kw)
    ls = orc.proxskip(g, b, estimator="lsvrg", **kw)
    sa = orc.proxskip(g, b, estimator="saga", **kw)
    assert np.array_equal(s[0], ls[0]) and np.array_equal(s[1], ls[1])
    scale = np.max(np.abs(s[0]))
    assert np.max(np.abs(sa[0] - s[0])) <= 1e-12 * scale
    assert s[3]["prox_calls"] == sa[3]["prox_calls"]


# ---------------------------------------------------------------------------------------------
# SAGA table (Eq. 4).
# ---------------------------------------------------------------------------------------------

def test_saga_table_state(orc):
    g, b = _problem(orc, seed=9)
    N = g.n_subsets
    gamma = 1.0 / (3.0 * orc.lipschitz(g, 300))
    K = 3 * N
    sub, coin = orc.sequences(13, 0, K, N, 0.3)
    sub = np.where(sub >= 2, sub - 2, sub).astype(np.int32)   # subsets 2 and 3 never drawn
    kw = dict(estimator="saga", gamma=gamma, p=0.3, alpha=1.0, fgp_inner=10, nonneg=True,
              sub=sub, coin=coin)
    x0 = np.zeros((1, g.ny, g.nx))
    xK, _, _, _, _, table, tsum = orc.proxskip(g, b, n_iters=K, return_table=True, **kw)
    # vbar = sum_i v_i
    assert np.max(np.abs(tsum - table.sum(axis=0))) <= 1e-12 * np.max(np.abs(tsum))
    # undrawn entries keep grad f_j(x_0)
    for j in (2, 3):
        assert np.array_equal(table[j], orc.grad_subset(g, x0, b, j))
    # the last drawn entry holds grad f_i at the iterate it was drawn at
    xK1 = orc.proxskip(g, b, n_iters=K - 1, sub=sub[:K - 1], coin=coin[:K - 1],
                       **{k: v for k, v in kw.items() if k not in ("sub", "coin")})[0]
    assert np.array_equal(table[sub[K - 1]], orc.grad_subset(g, xK1, b, int(sub[K - 1])))
    assert np.isfinite(xK).all()


def test_saga_first_step_is_full_gradient_step(orc):
    g, b = _problem(orc, seed=10)
    gamma = 0.3 / orc.lipschitz(g, 300)
    x0 = np.random.default_rng(1).random((1, g.ny, g.nx))
    x = orc.proxskip(g, b, estimator="saga", gamma=gamma, p=1.0, alpha=0.0, fgp_inner=0,
                     nonneg=False, plain=True, n_iters=1, sub=np.array([1], np.int32), x=x0)[0]
    x1 = x0 - gamma * orc.grad_full(g, x0, b)
    assert np.max(np.abs(x - x1)) <= 1e-13 * np.max(np.abs(x1))


@pytest.mark.parametrize("estimator", ["saga", "lsvrg"])
def test_trivial_prox_converges_to_least_squares(orc, estimator):
    # alpha = 0, no constraint, p = 1: the variance-reduced methods converge linearly to the
    # least-squares solution of a full-rank problem (SAGA with gamma = 1/(3L)).
    g = orc.Geometry(5, 5, n_angles=20, n_bins=9, n_subsets=4)
    M = _matrix(orc, g)
    lam = np.linalg.eigvalsh(M.T @ M)
    assert lam[0] > 1e-3 * lam[-1]
    b = np.random.default_rng(2).standard_normal((1, 20, 9))
    xstar = np.linalg.lstsq(M, b.ravel(), rcond=None)[0]
    gamma = 1.0 / (3.0 * lam[-1])
    x = orc.proxskip(g, b, estimator=estimator, gamma=gamma, p=1.0, alpha=0.0, fgp_inner=0,
                     nonneg=False, plain=True, n_epochs=10000, seed=3)[0]
    assert np.linalg.norm(x.ravel() - xstar) <= 1e-8 * np.linalg.norm(xstar)


# ---------------------------------------------------------------------------------------------
# FISTA.
# ---------------------------------------------------------------------------------------------

def test_fista_first_step_is_ista(orc):
    g, b = _problem(orc, N=1, seed=11)
    gamma = 1.0 / orc.lipschitz(g, 300)
    xf, df, _ = orc.fista(g, b, gamma=gamma, alpha=1.3, fgp_inner=20, n_iters=1, nonneg=True)
    xi, _, di, _, _ = orc.proxskip_svrg(g, b, gamma=gamma, p=1.0, alpha=1.3, fgp_inner=20,
                                        n_epochs=1, nonneg=True, plain=True)
    assert np.array_equal(xf, xi) and np.array_equal(df, di)


def test_fista_rate_bound(orc):
    # Beck & Teboulle (2009), Theorem 4.4 with step 1/L: F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k+1)^2
    g = orc.Geometry(5, 5, n_angles=20, n_bins=9, n_subsets=1)
    M = _matrix(orc, g)
    lam = np.linalg.eigvalsh(M.T @ M)
    L = lam[-1]
    b = np.random.default_rng(5).standard_normal((1, 20, 9))
    xstar = np.linalg.lstsq(M, b.ravel(), rcond=None)[0]
    Fstar = 0.5 * float(np.sum((M @ xstar - b.ravel()) ** 2))
    K = 400
    x, _, fval = orc.fista(g, b, gamma=1.0 / L, alpha=0.0, fgp_inner=0, n_iters=K, nonneg=False)
    k = np.arange(1, K + 1)                      # fval[k - 1] = F(x_k)
    bound = 2.0 * L * float(np.sum(xstar ** 2)) / (k + 1.0) ** 2
    assert np.all(fval - Fstar <= bound * (1 + 1e-12) + 1e-12 * Fstar)
    assert np.all(np.isfinite(x))
