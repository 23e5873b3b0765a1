"""ctypes declarations of the C ABI in include/proxskip.h (argument marshalling only).

The shared library is built in-tree (``paper_2602_09527_amd/libproxskip.so``) by ``build.py``.
Loading fails loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libproxskip.so")

PS_OK, PS_EINVAL, PS_ENOMEM, PS_EHIP, PS_EBUDGET, PS_ENONFINITE, PS_ECANCELLED, PS_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "PS_OK", -1: "PS_EINVAL", -2: "PS_ENOMEM", -3: "PS_EHIP", -4: "PS_EBUDGET",
                -5: "PS_ENONFINITE", -6: "PS_ECANCELLED", -7: "PS_EUNSUPPORTED"}
PS_F32, PS_F64 = 0, 1

# Every symbol include/proxskip.h declares.
EXPORTS = (
    "make_geometry", "free_geometry", "geometry_device_bytes", "geometry_upload", "subset_size",
    "geometry_get_plan", "geometry_set_plan", "geometry_autotune_workspace_bytes",
    "geometry_autotune",
    "project_workspace_bytes", "project_subset", "backproject_workspace_bytes",
    "backproject_subset", "tv_prox_workspace_bytes",
    "tv_prox_fgp", "proxskip_workspace_bytes", "proxskip_svrg_run", "solver_init",
    "solver_epochs", "solver_epochs_graph", "solver_steps", "solver_done", "solver_query",
    "solver_cancel",
    "solver_free", "sample_sequences", "sample_refresh_coins", "fista_workspace_bytes",
    "fista_run", "pdhg_workspace_bytes", "pdhg_run", "last_error_message",
    "proxskip_noalloc_max_bytes", "proxskip_svrg_run_noalloc",
    "kernel_timer_start", "kernel_timer_read", "kernel_timer_stop", "kernel_time_workspace_bytes",
    "kernel_time", "device_alloc", "device_free",
)
PS_EST_SVRG, PS_EST_LSVRG, PS_EST_SAGA = 0, 1, 2


class GeometryDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("n_angles", C.c_int32), ("angles", C.POINTER(C.c_double)),
        ("n_bins", C.c_int32), ("bin_width", C.c_double), ("det_offset", C.c_double),
        ("n_subsets", C.c_int32), ("dtype", C.c_int),
    ]


class Plan(C.Structure):
    _fields_ = [("proj_split_full", C.c_int32), ("proj_split_subset", C.c_int32),
                ("bp_groups_full", C.c_int32), ("bp_groups_subset", C.c_int32),
                ("bp_strip_full", C.c_int32), ("bp_strip_subset", C.c_int32),
                ("fgp_iters", C.c_int32), ("bp_method_full", C.c_int32),
                ("bp_method_subset", C.c_int32), ("bp_gather_rows", C.c_int32),
                ("fgp3d_chunk", C.c_int32), ("fgp_waves", C.c_int32), ("fgp_rows", C.c_int32),
                ("fgp3d_form", C.c_int32), ("bp_gather_split", C.c_int32),
                ("fgp_cols", C.c_int32),
                ("bp_gather_fused", C.c_int32)]


class SolverParams(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("p", C.c_double), ("alpha", C.c_double),
        ("fgp_inner", C.c_int32), ("nonneg", C.c_int32), ("n_epochs", C.c_int32),
        ("plain_prox_svrg", C.c_int32), ("seed", C.c_uint64), ("k0", C.c_int64),
        ("tol_rel_change", C.c_double), ("estimator", C.c_int32),
    ]


class SolverStats(C.Structure):
    _fields_ = [("epochs_done", C.c_int32), ("iters_done", C.c_int32),
                ("prox_calls", C.c_int32), ("last_rel_change", C.c_double)]


class NativeError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_lib = None


def load():
    """Load libproxskip.so (torch's HIP runtime must already be loaded: import torch first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2602_09527_amd.build` "
            "(or __graft_entry__.build()); there is no fallback implementation")
    import torch  # noqa: F401  -- the process must use torch's HIP runtime
    lib = C.CDLL(LIB_PATH)
    vp, sz, i32, i64, u64, d = C.c_void_p, C.c_size_t, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    st = C.c_int
    sig = {
        "make_geometry": (st, [C.POINTER(GeometryDesc), C.POINTER(vp)]),
        "free_geometry": (None, [vp]),
        "geometry_device_bytes": (sz, [vp]),
        "geometry_upload": (st, [vp, vp, sz, vp]),
        "subset_size": (i32, [vp, i32]),
        "geometry_get_plan": (st, [vp, C.POINTER(Plan)]),
        "geometry_set_plan": (st, [vp, C.POINTER(Plan)]),
        "geometry_autotune_workspace_bytes": (sz, [vp]),
        "geometry_autotune": (st, [vp, vp, sz, i32, vp, C.POINTER(Plan)]),
        "project_workspace_bytes": (sz, [vp, i32]),
        "project_subset": (st, [vp, i32, vp, vp, vp, sz, vp]),
        "backproject_workspace_bytes": (sz, [vp, i32]),
        "backproject_subset": (st, [vp, i32, vp, vp, i32, vp, sz, vp]),
        "tv_prox_workspace_bytes": (sz, [vp]),
        "tv_prox_fgp": (st, [vp, vp, vp, d, i32, i32, vp, vp, sz, vp]),
        "proxskip_workspace_bytes": (sz, [vp, C.POINTER(SolverParams)]),
        "proxskip_svrg_run": (st, [vp, vp, vp, vp, vp, C.POINTER(SolverParams),
                                   C.POINTER(SolverStats), vp, sz, vp]),
        "solver_init": (st, [vp, vp, vp, vp, vp, C.POINTER(SolverParams), vp, sz, C.POINTER(vp)]),
        "solver_epochs": (st, [C.POINTER(vp), i32, i32, vp]),
        "solver_steps": (st, [C.POINTER(vp), i32, i32, vp]),
        "solver_epochs_graph": (st, [C.POINTER(vp), i32, i32, vp]),
        "solver_done": (i32, [vp]),
        "solver_query": (st, [vp, C.POINTER(SolverStats)]),
        "solver_cancel": (st, [vp]),
        "solver_free": (None, [vp]),
        "sample_sequences": (st, [u64, i64, i64, i32, d, vp, vp]),
        "sample_refresh_coins": (st, [u64, i64, i64, i32, vp]),
        "fista_workspace_bytes": (sz, [vp]),
        "fista_run": (st, [vp, vp, vp, vp, vp, C.POINTER(d), d, d, i32, i32, i32, vp, sz, vp]),
        "pdhg_workspace_bytes": (sz, [vp]),
        "pdhg_run": (st, [vp, vp, vp, vp, vp, d, i32, i32, vp, sz, vp]),
        "last_error_message": (C.c_char_p, []),
        "proxskip_noalloc_max_bytes": (sz, []),
        "kernel_timer_start": (st, [C.c_uint32]),
        "kernel_timer_read": (st, [i32, C.POINTER(d), C.POINTER(i32)]),
        "kernel_timer_stop": (st, []),
        "kernel_time_workspace_bytes": (sz, [vp]),
        "kernel_time": (st, [vp, i32, i32, vp, sz, vp, C.POINTER(d)]),
        "proxskip_svrg_run_noalloc": (st, [vp, vp, vp, vp, vp, C.POINTER(SolverParams),
                                           C.POINTER(SolverStats), vp]),
        "device_alloc": (st, [sz, i32, C.POINTER(vp), C.POINTER(i32)]),
        "device_free": (st, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != PS_OK:
        msg = load().last_error_message()
        raise NativeError(status, where, msg.decode() if msg else "")
