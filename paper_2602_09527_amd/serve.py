"""Serving loop: reconstruction requests of mixed sizes, admitted by HBM budget and solved with
continuous batching on one GPU.

Each request is a 2D parallel-beam reconstruction (side N, A angles, B = 1.5 N bins) solved by
ProxSkip-SVRG until the relative change of an epoch falls below a tolerance, or an epoch cap.

Continuous batching.  The loop works in rounds.  Between rounds it admits requests that have
arrived, first come first served, while the HBM budget and the slot cap allow, and it retires
finished requests, freeing their memory.  A round advances every admitted request by a fixed
number of iterations with ``solver_steps``.  Each stage of an iteration is then one launch over
the work list of all admitted requests, so requests that arrive while others run share the
device with them.  Each request keeps x, h, the SVRG snapshot x~, its gradient and the FGP dual
resident in HBM from admission to completion.  Every request computes bit for bit what it
computes alone (the work-list kernels give each item its own geometry, buffers and plan).

The baseline serves the same trace one request at a time (each solved alone, in arrival order).
"""
from __future__ import annotations

import collections
import ctypes as C
import os
import dataclasses
import threading
import time

import numpy as np
import torch

from . import api, synth, workloads

PLANS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans_mi355x.json")


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float      # seconds after the start of the trace
    side: int           # image side N (N x N pixels)
    n_angles: int
    n_bins: int
    n_subsets: int
    seed: int           # phantom = seed, noise = seed + 1, subset/coin streams = seed + 2

    @property
    def key(self):
        return (self.side, self.n_angles, self.n_bins, self.n_subsets)


@dataclasses.dataclass
class ServeConfig:
    p: float = 0.1
    alpha: float = 0.01
    fgp_inner: int = 50
    tol: float = 1e-4              # stop at the first epoch end with relative change below tol
    max_epochs: int = 200          # epoch cap (a request that reaches it is reported unconverged)
    budget_bytes: int = 64 << 30   # HBM for admitted requests' buffers
    max_slots: int = 32            # admitted requests at most
    steps_per_round: int = 10      # iterations per round between admissions


def make_trace(n_requests: int, rate: float, seed: int, sides=workloads.SERVE_SIDES,
               angles=workloads.SERVE_ANGLES, subsets=None) -> list[Request]:
    """Poisson arrivals (exponential gaps with mean 1/rate), sides and angle counts uniform over
    the given sets, bins = 1.5 N, subset count by angle count."""
    subsets = subsets or workloads.SERVE_SUBSETS
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    side = rng.choice(np.asarray(sides), n_requests)
    ang = rng.choice(np.asarray(angles), n_requests)
    out = []
    for i in range(n_requests):
        N, A = int(side[i]), int(ang[i])
        out.append(Request(i, float(t[i]), N, A, (3 * N) // 2, int(subsets[A]), seed * 100003 + 7 * i))
    return out


class GeometryCache:
    """One geometry per request shape: device tables, autotuned launch plans and the step size
    gamma = 1/L (power method), all prepared once."""

    def __init__(self, device, power_iters: int = 30, tune: bool = True):
        self.device = torch.device(device)
        self.power_iters = power_iters
        self.tune = tune
        self._g = {}

    def get(self, r: Request):
        e = self._g.get(r.key)
        if e is None:
            g = api.Geometry(r.side, r.side, r.n_angles, r.n_bins, n_subsets=r.n_subsets,
                             device=self.device)
            if self.tune:
                # launch plans of this shape, before any workspace: stored ones when present
                api.autotune(g, reps=3, cache_path=PLANS_FILE, store=False)
            e = (g, api.lipschitz(g, self.power_iters))
            self._g[r.key] = e
        return e

    def warm(self, trace):
        for r in trace:
            self.get(r)


def request_sinogram(r: Request, device) -> torch.Tensor:
    """The request's data: exact line integrals of a seeded random-ellipse phantom plus 1%
    Gaussian noise, FP32, [1][A][B]."""
    ell = synth.random_ellipses(r.seed)
    s = synth.analytic_sinogram_torch(ell, r.side, r.side, r.n_angles, r.n_bins, device=device)
    return synth.gaussian_noise_torch(s, r.seed + 1).float()


def data_bank(trace, device) -> dict:
    """Every request's sinogram in pinned host memory (generated on the GPU beforehand)."""
    bank = {}
    for r in trace:
        bank[r.rid] = request_sinogram(r, device).cpu().pin_memory()
    return bank


def params_for(r: Request, cfg: ServeConfig, L: float) -> api.SolverParams:
    return api.SolverParams(gamma=1.0 / L, p=cfg.p, alpha=cfg.alpha, fgp_inner=cfg.fgp_inner,
                            n_epochs=cfg.max_epochs, nonneg=True, seed=r.seed + 2,
                            tol_rel_change=cfg.tol)


def footprint_bytes(g: api.Geometry, prm: api.SolverParams) -> int:
    """HBM a request holds while admitted: b, x, h, dual and the solver workspace."""
    p = prm.c()
    ws = g.lib.proxskip_workspace_bytes(g.handle, C.byref(p))
    elem = 4 if g.dtype == torch.float32 else 8
    return int(ws + elem * (g.nz * g.n_angles * g.n_bins + 2 * g.n + g.tv_dims * g.n))


def admit(trace_queue, used_bytes: int, n_active: int, now: float, cfg: ServeConfig, size_of):
    """Requests to admit now, first come first served: the head of the queue enters if it has
    arrived, a slot is free and its footprint fits what is left of the budget (used_bytes and
    n_active count everything already admitted); otherwise admission stops there.  A request
    larger than the whole budget can never be served and raises ValueError."""
    out = []
    used, slots = used_bytes, n_active
    for r in trace_queue:
        if r.arrival > now or slots >= cfg.max_slots:
            break
        need = size_of(r)
        if need > cfg.budget_bytes:
            raise ValueError(f"request {r.rid} needs {need} bytes, over the whole budget")
        if used + need > cfg.budget_bytes:
            break
        out.append(r)
        used += need
        slots += 1
    return out


@dataclasses.dataclass
class _Slot:
    req: Request
    solver: api.Solver
    nbytes: int
    admitted: float


def _result(req, solver, admitted, finished, keep):
    st = solver.query()
    res = dict(rid=req.rid, side=req.side, n_angles=req.n_angles, arrival=req.arrival,
               admitted=admitted, finished=finished, latency=finished - req.arrival,
               epochs=st["epochs_done"], converged=st["last_rel_change"] < solver.params.tol_rel_change,
               last_rel_change=st["last_rel_change"], prox_calls=st["prox_calls"])
    if keep is not None and req.rid in keep:
        res["x"] = solver.x.clone()
    return res


class _Budget:
    """HBM bytes and slots in use, shared by the size classes' loops."""

    def __init__(self):
        self.used = 0
        self.slots = 0
        self.lock = threading.Lock()


def _serve_class(trace, cfg, bank, geoms, keep, log, budget: _Budget, stream, t0, results, errors):
    """One size class: continuous batching in rounds on its own stream."""
    dev = geoms.device
    queue = collections.deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
    active: list[_Slot] = []
    sizes = {}

    def size_of(r):
        if r.rid not in sizes:
            g, L = geoms.get(r)
            sizes[r.rid] = footprint_bytes(g, params_for(r, cfg, L))
        return sizes[r.rid]

    try:
        with torch.cuda.stream(stream):
            rounds = 0
            while queue or active:
                now = time.perf_counter() - t0
                with budget.lock:
                    take = admit(queue, budget.used, budget.slots, now, cfg, size_of)
                    for r in take:
                        budget.used += size_of(r)
                        budget.slots += 1
                for r in take:
                    queue.popleft()
                    g, L = geoms.get(r)
                    b = bank[r.rid].to(dev, non_blocking=True)
                    s = api.Solver(g, b, params_for(r, cfg, L))
                    active.append(_Slot(r, s, size_of(r), time.perf_counter() - t0))
                if not active:
                    # idle: sleep until the next arrival, or poll while other classes hold the budget
                    wait = queue[0].arrival - (time.perf_counter() - t0)
                    time.sleep(wait if wait > 0 else 0.001)
                    continue
                api.run_steps([a.solver for a in active], cfg.steps_per_round, stream=stream)
                rounds += 1
                now = time.perf_counter() - t0
                still = []
                for a in active:
                    if a.solver.done():
                        results[a.req.rid] = _result(a.req, a.solver, a.admitted, now, keep)
                        a.solver.close()
                        with budget.lock:
                            budget.used -= a.nbytes
                            budget.slots -= 1
                    else:
                        still.append(a)
                active = still
                if log and rounds % 50 == 0:
                    log(f"serve: t={now:.1f}s active={len(active)} queued={len(queue)} done={len(results)}")
            stream.synchronize()
    except BaseException as e:  # reported by serve()
        errors.append(e)


def size_class(r: Request) -> int:
    """Requests are grouped by image side: each side runs on its own stream."""
    return r.side


def serve(trace, cfg: ServeConfig, bank: dict, geoms: GeometryCache, keep=None, log=None,
          classify=size_class):
    """Continuous batching over the trace (arrival times relative to the call).

    Requests are split into size classes (``classify``); each class runs its own batching loop on
    its own stream from its own host thread, so the kernels of small requests run beside those of
    large ones instead of waiting for their lockstep, and all classes share one HBM budget.
    Returns the per-request results in request order and the wall time."""
    geoms.warm(trace)
    groups = collections.defaultdict(list)
    for r in trace:
        groups[classify(r)].append(r)
    budget = _Budget()
    results, errors = {}, []
    streams = {k: torch.cuda.Stream(device=geoms.device) for k in groups}
    torch.cuda.synchronize(geoms.device)
    t0 = time.perf_counter()
    threads = [threading.Thread(target=_serve_class,
                                args=(groups[k], cfg, bank, geoms, keep, log, budget, streams[k], t0,
                                      results, errors))
               for k in sorted(groups)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return [results[r.rid] for r in trace], wall


def serve_sequential(trace, cfg: ServeConfig, bank: dict, geoms: GeometryCache, keep=None, log=None):
    """The same trace served one request at a time, each solved alone in arrival order."""
    dev = geoms.device
    results = {}
    t0 = time.perf_counter()
    for i, r in enumerate(sorted(trace, key=lambda r: (r.arrival, r.rid))):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        admitted = time.perf_counter() - t0
        g, L = geoms.get(r)
        b = bank[r.rid].to(dev, non_blocking=True)
        s = api.Solver(g, b, params_for(r, cfg, L))
        s.epochs(cfg.max_epochs)
        results[r.rid] = _result(r, s, admitted, time.perf_counter() - t0, keep)
        s.close()
        if log and (i + 1) % 50 == 0:
            log(f"serve-seq: {i + 1}/{len(trace)} at t={time.perf_counter() - t0:.1f}s")
    wall = time.perf_counter() - t0
    return [results[r.rid] for r in trace], wall


def summarize(results, wall: float) -> dict:
    lat = np.array([r["latency"] for r in results])
    return dict(requests=len(results), wall_s=round(wall, 3),
                throughput_req_s=round(len(results) / wall, 3),
                p50_latency_s=round(float(np.percentile(lat, 50)), 4),
                p99_latency_s=round(float(np.percentile(lat, 99)), 4),
                mean_latency_s=round(float(lat.mean()), 4),
                converged=int(sum(r["converged"] for r in results)),
                mean_epochs=round(float(np.mean([r["epochs"] for r in results])), 2))


def solve_alone(r: Request, cfg: ServeConfig, bank: dict, geoms: GeometryCache) -> torch.Tensor:
    """One request solved by itself (the reference for the alone-vs-mix invariance)."""
    g, L = geoms.get(r)
    b = bank[r.rid].to(geoms.device)
    s = api.Solver(g, b, params_for(r, cfg, L))
    s.epochs(cfg.max_epochs)
    x = s.x.clone()
    s.close()
    return x


__all__ = ["Request", "ServeConfig", "make_trace", "GeometryCache", "request_sinogram", "data_bank",
           "params_for", "footprint_bytes", "admit", "serve", "serve_sequential", "summarize",
           "solve_alone"]
