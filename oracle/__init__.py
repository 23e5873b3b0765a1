"""FP64 CPU oracle for ProxSkip-SVRG tomography -- test infrastructure only.

Thin ctypes wrapper over ``liboracle.so`` (built from ``oracle.c`` by ``oracle/build.py``).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package;
the product library never does, and this package never imports the product.

All arrays are float64 numpy arrays in the layouts stated in ``oracle.h``:
image ``[nz][ny][nx]``, sinogram ``[nz][A][B]``, subset sinogram ``[nz][a_i][B]``,
dual field ``[d][nz][ny][nx]`` with d = 2 for one slice and 3 otherwise.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Geom(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("n_angles", C.c_int), ("n_bins", C.c_int), ("n_subsets", C.c_int),
        ("du", C.c_double), ("off", C.c_double),
        ("angles", C.POINTER(C.c_double)),
    ]


class _Stats(C.Structure):
    _fields_ = [("epochs_done", C.c_int), ("iters_done", C.c_int), ("prox_calls", C.c_int),
                ("last_rel_change", C.c_double)]


_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_DN = C.c_void_p  # nullable double*
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # compile on first use (plain gcc, seconds)
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    G = C.POINTER(_Geom)
    sig = {
        "orc_subset_size": (C.c_int, [G, C.c_int]),
        "orc_project": (None, [G, C.c_int, _D, _D]),
        "orc_backproject": (None, [G, C.c_int, _D, _D]),
        "orc_project_rays": (None, [G, _D, C.c_int, _I, _I, _I, _D]),
        "orc_backproject_pixels": (None, [G, C.c_int, _D, C.c_int, _I, _I, _I, _D]),
        "orc_grad_subset": (None, [G, C.c_int, _D, _D, _D]),
        "orc_grad_full": (None, [G, _D, _D, _D]),
        "orc_data_fit": (C.c_double, [G, _D, _D]),
        "orc_lipschitz": (C.c_double, [G, C.c_int]),
        "orc_tv": (C.c_double, [C.c_int, C.c_int, C.c_int, _D]),
        "orc_tv_prox_fgp": (None, [C.c_int, C.c_int, C.c_int, _D, _D, C.c_double, C.c_int,
                                   C.c_int, _DN]),
        "orc_tv_prox_dpg": (None, [C.c_int, C.c_int, C.c_int, _D, _D, C.c_double, C.c_int,
                                   C.c_int, _DN]),
        "orc_splitmix64": (C.c_uint64, [C.c_uint64, C.c_uint64]),
        "orc_sequences": (None, [C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_double, _I, _U8]),
        "orc_proxskip_svrg": (C.c_int, [G, _D, _D, _D, _DN, C.c_double, C.c_double, C.c_double,
                                        C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_int64,
                                        C.c_double, C.POINTER(_Stats), _DN]),
        "orc_refresh_coins": (None, [C.c_uint64, C.c_int64, C.c_int64, C.c_int, _U8]),
        "orc_proxskip": (C.c_int, [G, _D, _D, _D, _DN, C.c_double, C.c_double, C.c_double,
                                   C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int64,
                                   _I, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(_Stats),
                                   _DN, _DN, _DN]),
        "orc_fista": (C.c_int, [G, _D, _D, _DN, C.c_double, C.c_double, C.c_int, C.c_int,
                                C.c_int, _DN]),
        "orc_pdhg": (C.c_int, [G, _D, _D, _D, _D, C.c_double, C.c_int, C.c_int]),
        "orc_num_threads": (C.c_int, []),
        "orc_set_num_threads": (None, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


@dataclasses.dataclass
class Geometry:
    """Parallel-beam geometry (see oracle.h for the conventions)."""
    nx: int
    ny: int
    n_angles: int
    n_bins: int
    n_subsets: int = 1
    nz: int = 1
    du: float = 1.0
    off: float = 0.0
    angles: np.ndarray | None = None

    def _c(self):
        ang = None
        if self.angles is not None:
            self._ang = np.ascontiguousarray(self.angles, dtype=np.float64)
            ang = self._ang.ctypes.data_as(C.POINTER(C.c_double))
        self._cg = _Geom(self.nx, self.ny, self.nz, self.n_angles, self.n_bins, self.n_subsets,
                         self.du, self.off, ang)
        return C.byref(self._cg)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def tv_dims(self) -> int:
        return 3 if self.nz > 1 else 2

    def subset_size(self, subset: int) -> int:
        return _load().orc_subset_size(self._c(), subset)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def project(g: Geometry, x, subset: int = -1) -> np.ndarray:
    x = _f64(x).reshape(g.nz, g.ny, g.nx)
    y = np.zeros((g.nz, g.subset_size(subset), g.n_bins))
    _load().orc_project(g._c(), subset, x, y)
    return y


def backproject(g: Geometry, y, subset: int = -1) -> np.ndarray:
    na = g.subset_size(subset)
    y = _f64(y).reshape(g.nz, na, g.n_bins)
    x = np.zeros((g.nz, g.ny, g.nx))
    _load().orc_backproject(g._c(), subset, y, x)
    return x


def project_rays(g: Geometry, x, zs, ks, us) -> np.ndarray:
    x = _f64(x).reshape(g.nz, g.ny, g.nx)
    zs, ks, us = (np.ascontiguousarray(a, dtype=np.int32) for a in (zs, ks, us))
    out = np.zeros(len(zs))
    _load().orc_project_rays(g._c(), x, len(zs), zs, ks, us, out)
    return out


def backproject_pixels(g: Geometry, y, zs, is_, js, subset: int = -1) -> np.ndarray:
    na = g.subset_size(subset)
    y = _f64(y).reshape(g.nz, na, g.n_bins)
    zs, is_, js = (np.ascontiguousarray(a, dtype=np.int32) for a in (zs, is_, js))
    out = np.zeros(len(zs))
    _load().orc_backproject_pixels(g._c(), subset, y, len(zs), zs, is_, js, out)
    return out


def grad_subset(g: Geometry, x, b, subset: int) -> np.ndarray:
    out = np.zeros((g.nz, g.ny, g.nx))
    _load().orc_grad_subset(g._c(), subset, _f64(x), _f64(b), out)
    return out


def grad_full(g: Geometry, x, b) -> np.ndarray:
    out = np.zeros((g.nz, g.ny, g.nx))
    _load().orc_grad_full(g._c(), _f64(x), _f64(b), out)
    return out


def data_fit(g: Geometry, x, b) -> float:
    return _load().orc_data_fit(g._c(), _f64(x), _f64(b))


def lipschitz(g: Geometry, iters: int = 500) -> float:
    return _load().orc_lipschitz(g._c(), iters)


def tv(z) -> float:
    z = _f64(z)
    nz, ny, nx = (1,) * (3 - z.ndim) + z.shape
    return _load().orc_tv(nx, ny, nz, z)


def _prox(fn, v, tau, n_inner, nonneg, dual):
    v = _f64(v)
    nz, ny, nx = (1,) * (3 - v.ndim) + v.shape
    z = np.zeros_like(v)
    dptr = None
    if dual is not None:
        assert dual.dtype == np.float64 and dual.flags.c_contiguous
        assert dual.size == (3 if nz > 1 else 2) * nx * ny * nz
        dptr = dual.ctypes.data
    getattr(_load(), fn)(nx, ny, nz, v, z, float(tau), int(n_inner), int(bool(nonneg)), dptr)
    return z


def tv_prox_fgp(v, tau, n_inner, nonneg=True, dual=None) -> np.ndarray:
    """z = prox_{tau (TV + I_C)}(v) by FGP; ``dual`` (float64, in/out) is the warm start."""
    return _prox("orc_tv_prox_fgp", v, tau, n_inner, nonneg, dual)


def tv_prox_dpg(v, tau, n_iter, nonneg=True, dual=None) -> np.ndarray:
    """Same prox by the unaccelerated dual projected gradient (an independent solver)."""
    return _prox("orc_tv_prox_dpg", v, tau, n_iter, nonneg, dual)


def splitmix64(seed: int, j: int) -> int:
    return _load().orc_splitmix64(seed, j)


def sequences(seed: int, k0: int, count: int, n_subsets: int, p: float):
    sub = np.zeros(max(count, 1), dtype=np.int32)
    coin = np.zeros(max(count, 1), dtype=np.uint8)
    _load().orc_sequences(seed, k0, count, n_subsets, float(p), sub, coin)
    return sub[:count], coin[:count]


def proxskip_svrg(g: Geometry, b, *, gamma, p, alpha, fgp_inner, n_epochs, nonneg=True,
                  plain=False, seed=0, k0=0, tol=0.0, x=None, h=None, dual=None):
    """Run ProxSkip-SVRG; returns (x, h, dual, stats dict, per-epoch relative changes).

    x, h, dual default to zeros (a fresh run); when given they are copied, not modified.
    """
    n = g.n
    x = np.zeros((g.nz, g.ny, g.nx)) if x is None else _f64(x).reshape(g.nz, g.ny, g.nx).copy()
    h = np.zeros((g.nz, g.ny, g.nx)) if h is None else _f64(h).reshape(g.nz, g.ny, g.nx).copy()
    dual = (np.zeros((g.tv_dims, g.nz, g.ny, g.nx)) if dual is None
            else _f64(dual).reshape(g.tv_dims, g.nz, g.ny, g.nx).copy())
    rel = np.zeros(max(n_epochs, 1))
    st = _Stats()
    rc = _load().orc_proxskip_svrg(g._c(), _f64(b), x, h, dual.ctypes.data, float(gamma),
                                   float(p), float(alpha), int(fgp_inner), int(bool(nonneg)),
                                   int(n_epochs), int(bool(plain)), int(seed), int(k0),
                                   float(tol), C.byref(st), rel.ctypes.data)
    if rc != 0:
        raise ValueError("orc_proxskip_svrg: invalid arguments")
    stats = dict(epochs_done=st.epochs_done, iters_done=st.iters_done,
                 prox_calls=st.prox_calls, last_rel_change=st.last_rel_change)
    assert x.size == n
    return x, h, dual, stats, rel[:st.epochs_done]


ESTIMATORS = {"svrg": 0, "lsvrg": 1, "saga": 2}


def refresh_coins(seed: int, k0: int, count: int, n_subsets: int) -> np.ndarray:
    """Loopless-SVRG refresh coins rho_k (probability 1/N), k = k0 .. k0 + count - 1."""
    out = np.zeros(max(count, 1), dtype=np.uint8)
    _load().orc_refresh_coins(seed, k0, count, n_subsets, out)
    return out[:count]


def proxskip(g: Geometry, b, *, estimator, gamma, p, alpha, fgp_inner, n_epochs=None,
             n_iters=None, nonneg=True, plain=False, seed=0, k0=0, tol=0.0, sub=None, coin=None,
             refresh=None, x=None, h=None, dual=None, return_table=False):
    """Algorithm 1 with the SVRG, loopless-SVRG or SAGA estimator ("svrg", "lsvrg", "saga").

    The random draws default to the seeded streams (sequences() and refresh_coins()) and may be
    given instead.  Returns (x, h, dual, stats dict, per-epoch relative changes) and, with
    return_table, also (table [N][nz][ny][nx], table_sum) of the SAGA estimator.
    """
    est = ESTIMATORS[estimator]
    N = g.n_subsets
    K = int(n_iters if n_iters is not None else n_epochs * N)
    if sub is None or coin is None:
        s_, c_ = sequences(seed, k0, K, N, p)
        sub = s_ if sub is None else sub
        coin = c_ if coin is None else coin
    if refresh is None and est == 1:
        refresh = refresh_coins(seed, k0, K, N)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    coin = np.ascontiguousarray(coin, dtype=np.uint8)
    refresh = None if refresh is None else np.ascontiguousarray(refresh, dtype=np.uint8)
    x = np.zeros((g.nz, g.ny, g.nx)) if x is None else _f64(x).reshape(g.nz, g.ny, g.nx).copy()
    h = np.zeros((g.nz, g.ny, g.nx)) if h is None else _f64(h).reshape(g.nz, g.ny, g.nx).copy()
    dual = (np.zeros((g.tv_dims, g.nz, g.ny, g.nx)) if dual is None
            else _f64(dual).reshape(g.tv_dims, g.nz, g.ny, g.nx).copy())
    rel = np.zeros(max(K // N + 1, 1))
    table = np.zeros((N, g.nz, g.ny, g.nx)) if (return_table and est == 2) else None
    tsum = np.zeros((g.nz, g.ny, g.nx)) if (return_table and est == 2) else None
    st = _Stats()
    rc = _load().orc_proxskip(g._c(), _f64(b), x, h, dual.ctypes.data, float(gamma), float(p),
                              float(alpha), int(fgp_inner), int(bool(nonneg)), int(bool(plain)),
                              est, int(k0), K, sub, coin.ctypes.data,
                              None if refresh is None else refresh.ctypes.data, float(tol),
                              C.byref(st), rel.ctypes.data,
                              None if table is None else table.ctypes.data,
                              None if tsum is None else tsum.ctypes.data)
    if rc != 0:
        raise ValueError("orc_proxskip: invalid arguments")
    stats = dict(epochs_done=st.epochs_done, iters_done=st.iters_done,
                 prox_calls=st.prox_calls, last_rel_change=st.last_rel_change)
    out = (x, h, dual, stats, rel[:st.epochs_done])
    return out + (table, tsum) if return_table else out


def fista(g: Geometry, b, *, gamma, alpha, fgp_inner, n_iters, nonneg=True, x=None, dual=None):
    """FISTA; returns (x, dual, objective f + alpha TV after each iteration)."""
    x = np.zeros((g.nz, g.ny, g.nx)) if x is None else _f64(x).reshape(g.nz, g.ny, g.nx).copy()
    dual = (np.zeros((g.tv_dims, g.nz, g.ny, g.nx)) if dual is None
            else _f64(dual).reshape(g.tv_dims, g.nz, g.ny, g.nx).copy())
    fval = np.zeros(max(n_iters, 1))
    rc = _load().orc_fista(g._c(), _f64(b), x, dual.ctypes.data, float(gamma), float(alpha),
                           int(fgp_inner), int(bool(nonneg)), int(n_iters), fval.ctypes.data)
    if rc != 0:
        raise ValueError("orc_fista: invalid arguments")
    return x, dual, fval[:n_iters]


def pdhg(g: Geometry, b, *, alpha, n_iters, nonneg=True, x=None, y1=None, y2=None):
    """Diagonally preconditioned PDHG for Eq. 5; returns (x, y1, y2) (copies of the inputs
    advanced by n_iters iterations; zeros when omitted)."""
    x = np.zeros((g.nz, g.ny, g.nx)) if x is None else _f64(x).reshape(g.nz, g.ny, g.nx).copy()
    y1 = (np.zeros((g.nz, g.n_angles, g.n_bins)) if y1 is None
          else _f64(y1).reshape(g.nz, g.n_angles, g.n_bins).copy())
    y2 = (np.zeros((g.tv_dims, g.nz, g.ny, g.nx)) if y2 is None
          else _f64(y2).reshape(g.tv_dims, g.nz, g.ny, g.nx).copy())
    rc = _load().orc_pdhg(g._c(), _f64(b), x, y1, y2, float(alpha), int(bool(nonneg)),
                          int(n_iters))
    if rc != 0:
        raise ValueError("orc_pdhg: invalid arguments")
    return x, y1, y2


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads for later oracle calls (results do not depend on it)."""
    _load().orc_set_num_threads(int(n))
