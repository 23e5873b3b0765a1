"""Python binding over the C ABI: torch tensors in, torch tensors out.

PyTorch only provides device memory and streams here; every step runs in the library's HIP
kernels.  Buffers follow the layouts of include/proxskip.h: image [nz][ny][nx], sinogram
[nz][A][B], subset sinogram [nz][a_i][B], dual [d][nz][ny][nx].
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _native as nat

_DTYPES = {torch.float32: nat.PS_F32, torch.float64: nat.PS_F64}


def _stream(device: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None else None)


# Workspaces of at least this many bytes come from the library's device_alloc (physically
# contiguous when the driver can provide it); smaller ones from torch's caching allocator.  A
# multi-GiB buffer built from small physical pieces slows the kernels that stream several of
# them at once (address translation), and only volume-sized workspaces reach this size.
CONTIGUOUS_MIN_BYTES = 1 << 30


class DeviceBuffer:
    """Device memory from device_alloc, used as a workspace: only its address and size are read
    (data_ptr, numel, like a uint8 tensor's).  Released with device_free -- which first waits for
    the device's queued work -- when the last reference goes."""

    def __init__(self, nbytes: int, device: torch.device):
        self.lib = nat.load()
        p, contig = C.c_void_p(), C.c_int32()
        nat.check(self.lib.device_alloc(int(nbytes), int(device.index), C.byref(p), C.byref(contig)),
                  "device_alloc")
        self.ptr, self.nbytes, self.contiguous = p.value, int(nbytes), bool(contig.value)

    def data_ptr(self) -> int:
        return self.ptr

    def numel(self) -> int:
        return self.nbytes

    def __del__(self):
        p = getattr(self, "ptr", None)
        if p:
            self.ptr = None
            try:
                self.lib.device_free(C.c_void_p(p))
            except Exception:   # interpreter shutdown
                pass


def workspace_buffer(nbytes: int, device: torch.device):
    """A workspace of `nbytes` on `device` (see CONTIGUOUS_MIN_BYTES)."""
    if nbytes >= CONTIGUOUS_MIN_BYTES:
        return DeviceBuffer(nbytes, device)
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Geometry:
    """Parallel-beam geometry with its per-angle tables resident on ``device``."""

    def __init__(self, nx: int, ny: int, n_angles: int, n_bins: int, n_subsets: int = 1,
                 nz: int = 1, bin_width: float = 1.0, det_offset: float = 0.0,
                 angles=None, dtype: torch.dtype = torch.float32, device="cuda"):
        if dtype not in _DTYPES:
            raise TypeError(f"dtype must be float32 or float64, got {dtype}")
        self.lib = nat.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n_angles, self.n_bins, self.n_subsets = int(n_angles), int(n_bins), int(n_subsets)
        self.bin_width, self.det_offset = float(bin_width), float(det_offset)
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on the GPU only; device must be a cuda device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._angles = None
        ang_ptr = None
        if angles is not None:
            self._angles = np.ascontiguousarray(angles, dtype=np.float64)
            if self._angles.shape != (self.n_angles,):
                raise ValueError("angles must have n_angles entries")
            ang_ptr = self._angles.ctypes.data_as(C.POINTER(C.c_double))
        desc = nat.GeometryDesc(self.nx, self.ny, self.nz, self.n_angles, ang_ptr, self.n_bins,
                                self.bin_width, self.det_offset, self.n_subsets, _DTYPES[dtype])
        h = C.c_void_p()
        nat.check(self.lib.make_geometry(C.byref(desc), C.byref(h)), "make_geometry")
        self.handle = h
        nbytes = self.lib.geometry_device_bytes(h)
        with torch.cuda.device(self.device):
            self._tables = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
            nat.check(self.lib.geometry_upload(h, _ptr(self._tables), nbytes, _stream(self.device)),
                      "geometry_upload")
        self._ws = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                self.lib.free_geometry(h)
            except Exception:
                pass
            self.handle = None

    # -- shapes -----------------------------------------------------------------------------
    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def tv_dims(self) -> int:
        return 3 if self.nz > 1 else 2

    @property
    def image_shape(self):
        return (self.nz, self.ny, self.nx)

    def subset_size(self, subset: int) -> int:
        a = self.lib.subset_size(self.handle, int(subset))
        if a < 0:
            raise ValueError(f"subset {subset} out of range")
        return a

    def sino_shape(self, subset: int = -1):
        return (self.nz, self.subset_size(subset), self.n_bins)

    def dual_shape(self):
        return (self.tv_dims, self.nz, self.ny, self.nx)

    # -- launch plan ------------------------------------------------------------------------
    @property
    def key(self) -> str:
        """Shape key of this geometry (for caches of tuned plans)."""
        dt = "f64" if self.dtype == torch.float64 else "f32"
        return (f"{self.nx}x{self.ny}x{self.nz}_a{self.n_angles}_b{self.n_bins}_n{self.n_subsets}"
                f"_w{self.bin_width:g}_o{self.det_offset:g}_{dt}" + ("_custom" if self._angles is not None else ""))

    def get_plan(self) -> dict:
        """The launch plan in effect (automatic choices filled in)."""
        p = nat.Plan()
        nat.check(self.lib.geometry_get_plan(self.handle, C.byref(p)), "geometry_get_plan")
        return {f: getattr(p, f) for f, _ in nat.Plan._fields_}

    def set_plan(self, plan: dict) -> None:
        """Override launch-plan fields (0 = automatic); set before sizing workspaces."""
        p = nat.Plan(**{f: int(plan.get(f, 0)) for f, _ in nat.Plan._fields_})
        nat.check(self.lib.geometry_set_plan(self.handle, C.byref(p)), "geometry_set_plan")
        self._ws = {}

    # -- buffers ----------------------------------------------------------------------------
    def check(self, t: torch.Tensor, shape, what: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{what} is on {t.device}, geometry is on {self.device}")
        if t.dtype != self.dtype:
            raise TypeError(f"{what} has dtype {t.dtype}, geometry uses {self.dtype}")
        # contiguity first: a reshape of a strided tensor would hand the kernels a copy, and an
        # in/out buffer (x, h, dual, out) would then be updated in the copy, not in the caller's
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if tuple(t.shape) != tuple(shape):
            if t.numel() != math.prod(shape):
                raise ValueError(f"{what} must have shape {tuple(shape)}")
            t = t.view(shape)   # a view of the same memory, never a copy
        return t

    def workspace(self, key, nbytes: int) -> torch.Tensor | None:
        if nbytes == 0:
            return None
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = workspace_buffer(nbytes, self.device)
            self._ws[key] = ws
        return ws

    def empty_image(self):
        return torch.empty(self.image_shape, dtype=self.dtype, device=self.device)

    def zeros_image(self):
        return torch.zeros(self.image_shape, dtype=self.dtype, device=self.device)


def project(g: Geometry, x: torch.Tensor, subset: int = -1, out: torch.Tensor | None = None):
    """y = A_i x (subset = -1: all angles)."""
    x = g.check(x, g.image_shape, "x")
    shape = g.sino_shape(subset)
    y = torch.empty(shape, dtype=g.dtype, device=g.device) if out is None else g.check(out, shape, "out")
    nbytes = g.lib.project_workspace_bytes(g.handle, int(subset))
    ws = g.workspace(("proj", shape[1]), nbytes)
    nat.check(g.lib.project_subset(g.handle, int(subset), _ptr(x), _ptr(y), _ptr(ws), nbytes,
                                   _stream(g.device)), "project_subset")
    return y


def backproject(g: Geometry, y: torch.Tensor, subset: int = -1, out: torch.Tensor | None = None,
                accumulate: bool = False):
    """x = A_i^T y, or out += A_i^T y with accumulate=True."""
    y = g.check(y, g.sino_shape(subset), "y")
    if accumulate and out is None:
        raise ValueError("accumulate=True needs out")
    x = g.empty_image() if out is None else g.check(out, g.image_shape, "out")
    nbytes = g.lib.backproject_workspace_bytes(g.handle, int(subset))
    ws = g.workspace(("bp", int(subset) if subset < 0 else 0), nbytes)
    nat.check(g.lib.backproject_subset(g.handle, int(subset), _ptr(y), _ptr(x), int(bool(accumulate)),
                                       _ptr(ws), nbytes, _stream(g.device)), "backproject_subset")
    return x


def tv_prox(g: Geometry, v: torch.Tensor, tau: float, n_inner: int, nonneg: bool = True,
            dual: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """z = prox_{tau (TV + I_C)}(v) by FGP; ``dual`` (in/out) is the warm start."""
    v = g.check(v, g.image_shape, "v")
    z = g.empty_image() if out is None else g.check(out, g.image_shape, "out")
    if dual is not None:
        dual = g.check(dual, g.dual_shape(), "dual")
    nbytes = g.lib.tv_prox_workspace_bytes(g.handle)
    ws = g.workspace("fgp", nbytes)
    nat.check(g.lib.tv_prox_fgp(g.handle, _ptr(v), _ptr(z), float(tau), int(n_inner), int(bool(nonneg)),
                                _ptr(dual), _ptr(ws), nbytes, _stream(g.device)), "tv_prox_fgp")
    return z


ESTIMATORS = {"svrg": nat.PS_EST_SVRG, "lsvrg": nat.PS_EST_LSVRG, "saga": nat.PS_EST_SAGA}


@dataclasses.dataclass
class SolverParams:
    """Algorithm 1 parameters (gamma, p), TV weight, FGP inner iterations, stopping rule, and
    the gradient estimator: "svrg" (ProxSVRGSkip), "lsvrg" (ProxLSVRGSkip) or "saga"
    (ProxSAGASkip)."""
    gamma: float
    p: float
    alpha: float
    fgp_inner: int
    n_epochs: int
    nonneg: bool = True
    plain_prox_svrg: bool = False
    seed: int = 0
    k0: int = 0
    tol_rel_change: float = 0.0
    estimator: str = "svrg"

    def c(self) -> nat.SolverParams:
        return nat.SolverParams(float(self.gamma), float(self.p), float(self.alpha),
                                int(self.fgp_inner), int(bool(self.nonneg)), int(self.n_epochs),
                                int(bool(self.plain_prox_svrg)), int(self.seed), int(self.k0),
                                float(self.tol_rel_change), int(ESTIMATORS[self.estimator]))


def _stats(s: nat.SolverStats) -> dict:
    return dict(epochs_done=s.epochs_done, iters_done=s.iters_done, prox_calls=s.prox_calls,
                last_rel_change=s.last_rel_change)


def solve(g: Geometry, b: torch.Tensor, params: SolverParams, x=None, h=None, dual=None):
    """Run Algorithm 1 with params.estimator; x, h, dual (in/out, zeros if omitted) are updated
    in place.

    Returns (x, h, dual, stats)."""
    b = g.check(b, (g.nz, g.n_angles, g.n_bins), "b")
    x = g.zeros_image() if x is None else g.check(x, g.image_shape, "x")
    h = g.zeros_image() if h is None else g.check(h, g.image_shape, "h")
    dual = (torch.zeros(g.dual_shape(), dtype=g.dtype, device=g.device) if dual is None
            else g.check(dual, g.dual_shape(), "dual"))
    prm = params.c()
    nbytes = g.lib.proxskip_workspace_bytes(g.handle, C.byref(prm))
    ws = workspace_buffer(nbytes, g.device)
    st = nat.SolverStats()
    nat.check(g.lib.proxskip_svrg_run(g.handle, _ptr(b), _ptr(x), _ptr(h), _ptr(dual), C.byref(prm),
                                      C.byref(st), _ptr(ws), nbytes, _stream(g.device)),
              "proxskip_svrg_run")
    return x, h, dual, _stats(st)


def solve_noalloc(g: Geometry, b: torch.Tensor, params: SolverParams, x=None, h=None, dual=None):
    """``solve`` without a workspace: the library's fixed per-GPU scratch array holds the solver's
    work buffers (proxskip_svrg_run_noalloc; at most proxskip_noalloc_max_bytes() of them, a fixed
    number of epochs, and calls on one GPU must not overlap).  Allocates nothing on the device
    beyond x, h, dual when they are omitted.

    Returns (x, h, dual, stats)."""
    b = g.check(b, (g.nz, g.n_angles, g.n_bins), "b")
    x = g.zeros_image() if x is None else g.check(x, g.image_shape, "x")
    h = g.zeros_image() if h is None else g.check(h, g.image_shape, "h")
    dual = (torch.zeros(g.dual_shape(), dtype=g.dtype, device=g.device) if dual is None
            else g.check(dual, g.dual_shape(), "dual"))
    prm = params.c()
    st = nat.SolverStats()
    with torch.cuda.device(g.device):
        nat.check(g.lib.proxskip_svrg_run_noalloc(g.handle, _ptr(b), _ptr(x), _ptr(h), _ptr(dual),
                                                  C.byref(prm), C.byref(st), _stream(g.device)),
                  "proxskip_svrg_run_noalloc")
    return x, h, dual, _stats(st)


KERNEL_CLASSES = {"backproject_subset": 1, "backproject_full": 2, "project_subset": 3,
                  "project_full": 4, "backproject_combine": 5, "project_reduce": 6,
                  "backproject_gather": 7, "fgp2d": 8, "fgp3d": 9}


class KernelTimer:
    """GPU time of chosen kernel classes inside the calls made while it is active (HIP events
    recorded by the library around each launch of those classes):

        with api.KernelTimer(["backproject_subset"]) as kt:
            solver.epochs(5)
        ms, launches = kt.result("backproject_subset")
    """

    def __init__(self, classes):
        self.lib = nat.load()
        self.classes = list(classes)
        self.mask = 0
        for c in self.classes:
            self.mask |= 1 << KERNEL_CLASSES[c]

    def __enter__(self):
        nat.check(self.lib.kernel_timer_start(self.mask), "kernel_timer_start")
        return self

    def __exit__(self, *exc):
        nat.check(self.lib.kernel_timer_stop(), "kernel_timer_stop")
        return False

    def result(self, cls: str):
        """(summed milliseconds, launches) of the class."""
        ms, n = C.c_double(), C.c_int32()
        nat.check(self.lib.kernel_timer_read(KERNEL_CLASSES[cls], C.byref(ms), C.byref(n)),
                  "kernel_timer_read")
        return ms.value, n.value


def kernel_time(g: Geometry, cls: str, reps: int = 100) -> float:
    """Average GPU time (microseconds) of one launch of one projector or backprojector kernel
    class alone on this geometry (HIP events around `reps` back-to-back launches on the current
    stream; see kernel_time in include/proxskip.h)."""
    nbytes = g.lib.kernel_time_workspace_bytes(g.handle)
    ws = workspace_buffer(nbytes, g.device)
    us = C.c_double()
    nat.check(g.lib.kernel_time(g.handle, KERNEL_CLASSES[cls], int(reps), _ptr(ws), nbytes,
                                _stream(g.device), C.byref(us)), "kernel_time")
    return us.value


class Solver:
    """Resumable ProxSkip-SVRG handle: owns its state tensors and workspace."""

    def __init__(self, g: Geometry, b: torch.Tensor, params: SolverParams, x=None, h=None,
                 dual=None):
        self.g = g
        self.b = g.check(b, (g.nz, g.n_angles, g.n_bins), "b")
        self.x = g.zeros_image() if x is None else g.check(x, g.image_shape, "x")
        self.h = g.zeros_image() if h is None else g.check(h, g.image_shape, "h")
        self.dual = (torch.zeros(g.dual_shape(), dtype=g.dtype, device=g.device) if dual is None
                     else g.check(dual, g.dual_shape(), "dual"))
        self.params = params
        self._prm = params.c()
        nbytes = g.lib.proxskip_workspace_bytes(g.handle, C.byref(self._prm))
        self.ws = workspace_buffer(nbytes, g.device)
        h_ = C.c_void_p()
        nat.check(g.lib.solver_init(g.handle, _ptr(self.b), _ptr(self.x), _ptr(self.h),
                                    _ptr(self.dual), C.byref(self._prm), _ptr(self.ws), nbytes,
                                    C.byref(h_)), "solver_init")
        self.handle = h_

    def epochs(self, n: int, stream=None, graph: bool = False):
        run_epochs([self], n, stream, graph=graph)

    def done(self) -> bool:
        """True once the handle will not advance any further (no synchronisation)."""
        return self.g.lib.solver_done(self.handle) == 1

    def query(self) -> dict:
        st = nat.SolverStats()
        nat.check(self.g.lib.solver_query(self.handle, C.byref(st)), "solver_query")
        return _stats(st)

    def cancel(self):
        nat.check(self.g.lib.solver_cancel(self.handle), "solver_cancel")

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.g.lib.solver_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_epochs(solvers, n_epochs: int, stream=None, graph: bool = False):
    """Run ``n_epochs`` more epochs of every solver, batched in lockstep (one launch per stage
    over all solvers); each solver's result is bit for bit its result alone.  graph=True issues
    every epoch round as a captured HIP graph (solver_epochs_graph)."""
    if not solvers:
        return
    arr = (C.c_void_p * len(solvers))(*[s.handle for s in solvers])
    dev = solvers[0].g.device
    st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(dev)
    lib = solvers[0].g.lib
    if graph:
        nat.check(lib.solver_epochs_graph(arr, len(solvers), int(n_epochs), st), "solver_epochs_graph")
    else:
        nat.check(lib.solver_epochs(arr, len(solvers), int(n_epochs), st), "solver_epochs")


def run_steps(solvers, n_steps: int, stream=None):
    """Advance every solver by up to ``n_steps`` iterations in lockstep (batched launches)."""
    if not solvers:
        return
    arr = (C.c_void_p * len(solvers))(*[s.handle for s in solvers])
    dev = solvers[0].g.device
    st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(dev)
    nat.check(solvers[0].g.lib.solver_steps(arr, len(solvers), int(n_steps), st), "solver_steps")


def sample_sequences(seed: int, k0: int, count: int, n_subsets: int, p: float):
    """The library's host-side subset and coin streams (int32, uint8 numpy arrays)."""
    lib = nat.load()
    sub = np.zeros(max(count, 1), dtype=np.int32)
    coin = np.zeros(max(count, 1), dtype=np.uint8)
    nat.check(lib.sample_sequences(int(seed), int(k0), int(count), int(n_subsets), float(p),
                                   sub.ctypes.data_as(C.c_void_p), coin.ctypes.data_as(C.c_void_p)),
              "sample_sequences")
    return sub[:count], coin[:count]


def sample_refresh_coins(seed: int, k0: int, count: int, n_subsets: int):
    """The library's loopless-SVRG refresh coins (uint8 numpy array)."""
    lib = nat.load()
    out = np.zeros(max(count, 1), dtype=np.uint8)
    nat.check(lib.sample_refresh_coins(int(seed), int(k0), int(count), int(n_subsets),
                                       out.ctypes.data_as(C.c_void_p)), "sample_refresh_coins")
    return out[:count]


class Fista:
    """FISTA with the full gradient and the TV prox (resumable: each call continues the run).

    State: x, the extrapolated point y, the FGP dual and the momentum scalar t (zeros / x_0 / 1
    for a fresh run).  Stream-ordered on the current stream."""

    def __init__(self, g: Geometry, b: torch.Tensor, gamma: float, alpha: float, fgp_inner: int,
                 nonneg: bool = True, x=None, dual=None):
        self.g = g
        self.b = g.check(b, (g.nz, g.n_angles, g.n_bins), "b")
        self.x = g.zeros_image() if x is None else g.check(x, g.image_shape, "x")
        self.y = self.x.clone()
        self.dual = (torch.zeros(g.dual_shape(), dtype=g.dtype, device=g.device) if dual is None
                     else g.check(dual, g.dual_shape(), "dual"))
        self.t = C.c_double(1.0)
        self.gamma, self.alpha, self.fgp_inner, self.nonneg = gamma, alpha, fgp_inner, nonneg
        self.nbytes = g.lib.fista_workspace_bytes(g.handle)
        self.ws = workspace_buffer(self.nbytes, g.device)

    def run(self, n_iters: int):
        g = self.g
        nat.check(g.lib.fista_run(g.handle, _ptr(self.b), _ptr(self.x), _ptr(self.y),
                                  _ptr(self.dual), C.byref(self.t), float(self.gamma),
                                  float(self.alpha), int(self.fgp_inner), int(bool(self.nonneg)),
                                  int(n_iters), _ptr(self.ws), self.nbytes, _stream(g.device)),
                  "fista_run")
        return self


def fista(g: Geometry, b: torch.Tensor, gamma: float, alpha: float, fgp_inner: int, n_iters: int,
          nonneg: bool = True, x=None, dual=None):
    """A fresh FISTA run of n_iters iterations from x (zeros if omitted); x and dual are
    updated in place.  Returns (x, dual)."""
    f = Fista(g, b, gamma, alpha, fgp_inner, nonneg=nonneg, x=x, dual=dual).run(n_iters)
    return f.x, f.dual


def pdhg(g: Geometry, b: torch.Tensor, alpha: float, n_iters: int, nonneg: bool = True, x=None,
         y1=None, y2=None):
    """Reference solution of Eq. 5 by preconditioned PDHG; (x, y1, y2) (zeros if omitted) are
    advanced n_iters iterations in place and returned.  Stream-ordered on the current stream."""
    b = g.check(b, (g.nz, g.n_angles, g.n_bins), "b")
    x = g.zeros_image() if x is None else g.check(x, g.image_shape, "x")
    y1 = (torch.zeros((g.nz, g.n_angles, g.n_bins), dtype=g.dtype, device=g.device) if y1 is None
          else g.check(y1, (g.nz, g.n_angles, g.n_bins), "y1"))
    y2 = (torch.zeros(g.dual_shape(), dtype=g.dtype, device=g.device) if y2 is None
          else g.check(y2, g.dual_shape(), "y2"))
    nbytes = g.lib.pdhg_workspace_bytes(g.handle)
    ws = g.workspace("pdhg", nbytes)
    nat.check(g.lib.pdhg_run(g.handle, _ptr(b), _ptr(x), _ptr(y1), _ptr(y2), float(alpha),
                             int(bool(nonneg)), int(n_iters), _ptr(ws), nbytes, _stream(g.device)),
              "pdhg_run")
    return x, y1, y2


def autotune(g: Geometry, reps: int = 5, cache_path: str | None = None, store: bool = True,
             tune_missing: bool = True) -> dict:
    """Time candidate launch plans on the device and keep the fastest (see geometry_autotune).

    With ``cache_path`` (a JSON file keyed by Geometry.key), a plan stored for the same geometry
    is used as is; otherwise the geometry is tuned (unless tune_missing is False, which keeps
    the automatic plan) and, with ``store``, the new plan is added to the file."""
    import json
    import os
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if g.key in cache:
            g.set_plan(cache[g.key])
            return g.get_plan()
    if not tune_missing:
        return g.get_plan()
    nbytes = g.lib.geometry_autotune_workspace_bytes(g.handle)
    ws = workspace_buffer(nbytes, g.device)
    p = nat.Plan()
    nat.check(g.lib.geometry_autotune(g.handle, _ptr(ws), nbytes, int(reps), _stream(g.device),
                                      C.byref(p)), "geometry_autotune")
    del ws
    g._ws = {}
    plan = {f: getattr(p, f) for f, _ in nat.Plan._fields_}
    if cache_path and store:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[g.key] = plan
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return plan


def lipschitz(g: Geometry, iters: int = 100, seed: int = 0) -> float:
    """L = lambda_max(A^T A) by the power method on the GPU (step size gamma = 1/L).

    Starts from the all-ones image (A^T A is entrywise non-negative, so it overlaps the top
    eigenvector) and returns the last Rayleigh quotient, computed in float64."""
    v = torch.ones(g.image_shape, dtype=g.dtype, device=g.device)
    v /= torch.linalg.vector_norm(v.double()).to(g.dtype)
    lam = 0.0
    for _ in range(iters):
        w = backproject(g, project(g, v))
        lam = float(torch.sum(v.double() * w.double()))
        nrm = torch.linalg.vector_norm(w.double())
        if float(nrm) == 0.0:
            break
        v = (w.double() / nrm).to(g.dtype)
    return lam
