"""Benchmark: ProxSkip-SVRG epochs per second on one MI355X.

Workload (default): the single 512^2 solve -- 720 angles x 768 bins, 20 interleaved subsets,
p = 0.1, alpha = 0.005, 50 warm-started FGP iterations per prox, seeded random-ellipse phantom
with exact line-integral data and 1% Gaussian noise.  One step = one epoch (N = 20 iterations:
the SVRG snapshot with its full projection/backprojection, 20 subset projection/backprojection
pairs with the fused SVRG/ProxSkip update, and the FGP prox on the coin flips that hit).

Prints one JSON line.  Besides the timed epochs it reports:
  roofline      the kernel class with the most GPU time per epoch (per-launch HIP events on the
                launching stream over a second pass of the solve), rated on one launch timed
                alone: algorithmic lane operations per second against the VALU issue peak, and
                the HBM bytes per launch from the committed rocprofv3 counter summary (null once
                the kernel source has changed);
  kernel_time_per_epoch  that per-class breakdown of the epoch;
  kernels       each operator's rate in samples/s, lane operations/s and algorithmic GB/s;
  sweep         epochs/s and prox calls at p in {1, 0.1, 0.02}, non-skipped ProxSVRG, ProxLSVRGSkip
                and ProxSAGASkip at p = 0.1, and iterations/s (one data pass each) of ISTA,
                deterministic ProxSkip (p = 0.1) and FISTA;
  time_to_eps   the paper's protocol: data passes and seconds until ||x - x*||^2/||x*||^2 < 1e-3
                and 1e-5 for the methods of the sweep, x* from preconditioned PDHG;
  batch         64 independent 128^2 solves batched in lockstep against one after another;
  serving       a Poisson trace of mixed-size requests with continuous batching against one
                request at a time (p50/p99 latency, throughput);
  cpu_baseline  the FP64 oracle timed on the host cores over a bounded sample of the same solve;
  parity        the GPU iterate against the oracle's after that sample;
  volume        the 256 x 1024^2 volume with 3D TV as a bounded leg (1 warm-up and 2 timed epochs
                unless --volume-epochs says otherwise): per-operator times with the stored and the
                automatic plan, one epoch eager against a HIP graph, the oracle's per-operator
                times on a few slices.

--volume times the 256 x 1024^2 volume instead (5 epochs after 1 warm-up unless --steps and
--warmup say otherwise); --calibrate-copy runs only a plain device copy
of known size (for scaling the HBM byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "epochs/s to 1e-4 rel-err vs oracle; projector HBM GB/s; p50/p99 recon latency"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane operations per second
# (one non-packed FP32 or integer operation per lane per cycle; packed FP32 is not used).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic lane operations per interpolation sample (one ray crossing one row or column):
#   projector:     position step, floor, weight, v1 - v0, fused multiply-add, accumulate  = 6
#   backprojector: position step, floor, weight, w y, y - w y, two accumulations        = 7
OPS_PROJECT = 6
OPS_BACKPROJECT = 7
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_2d-512-a720.txt")
# launch plans tuned once on an MI355X (python -m paper_2602_09527_amd.tune_plans); a geometry
# missing from the file is tuned on the spot
PLANS_FILE = os.path.join(ROOT, "paper_2602_09527_amd", "plans_mi355x.json")


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class (e.g. backproject_subset) from the committed
    rocprofv3 counter summary, or None when the summary has no line for it or the kernel's
    source differs from the one the counters were taken on."""
    import hashlib
    try:
        lines = [l for l in open(TRAFFIC_FILE) if l.startswith("traffic:")]
    except OSError:
        return None
    for line in lines:
        kv = dict(tok.split("=", 1) for tok in line.split()[1:])
        if kv.get("class") != kernel_class:
            continue
        src = os.path.join(ROOT, "paper_2602_09527_amd", "csrc", kv.get("source", ""))
        try:
            with open(src, "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != kv.get("source_sha256"):
                    return None
        except OSError:
            return None
        return (float(kv["fetch_kib"]) * float(kv["fetch_factor"]) +
                float(kv["write_kib"]) * float(kv["write_factor"])) * 1024.0
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed epochs (200; 5 with --volume)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed epochs (5; 1 with --volume)")
    ap.add_argument("--p", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--cpu-epochs", type=int, default=12,
                    help="epochs of the oracle sample (about 10 s on 16 host threads)")
    ap.add_argument("--no-eps", action="store_true",
                    help="skip the time-to-epsilon comparison against the PDHG reference x*")
    ap.add_argument("--ref-iters", type=int, default=100000,
                    help="PDHG iterations of the reference x* (the paper uses 2e5)")
    ap.add_argument("--eps-passes", type=int, default=200, help="data passes per method at most")
    ap.add_argument("--subset-sweep", action="store_true",
                    help="also run ProxSVRGSkip (p = 0.3) against ProxSVRG for N in {10, 50, 100, "
                         "200, 400} subsets on the time-to-epsilon problem (about a minute)")
    ap.add_argument("--eps-alpha", type=float, default=50.0,
                    help="TV weight of the time-to-epsilon problem: 50 makes 1e-5 reachable in 200 "
                         "data passes; at the workload's 0.005 the problem is nearly unregularised "
                         "least squares and no method gets below 1e-3 in 200 passes")
    ap.add_argument("--no-oracle-extra", action="store_true",
                    help="skip the oracle's 1-thread run and its timings on the other workloads")
    ap.add_argument("--no-volume", action="store_true",
                    help="skip the bounded leg on the 256 x 1024^2 volume")
    ap.add_argument("--volume-epochs", type=int, default=2,
                    help="timed epochs of the volume leg (after one warm-up)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the bounded serving trace")
    ap.add_argument("--serve-cap", type=int, default=200,
                    help="epoch cap per served request (each stops earlier at 1e-4 relative change)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrivals per second")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (for HBM counter scaling)")
    ap.add_argument("--volume", action="store_true",
                    help="time the 256 x 1024^2 volume workload (1800 x 1448, 30 subsets) instead")
    ap.add_argument("--volume-ops", action="store_true",
                    help="only run one subset projection, one subset backprojection and a 10-iteration "
                         "3D prox on the volume geometry with random inputs (for counter collection)")
    ap.add_argument("--solve", default=None, metavar="WORKLOAD",
                    help="only time --steps epochs of one 2D workload's solve after --warmup "
                         "(2d-128-a180 or 2d-512-a720; a short program for kernel traces)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 5 if args.volume else 200
    if args.warmup is None:
        args.warmup = 1 if args.volume else 5
    return args


def stored_L(w):
    path = os.path.join(ROOT, "tests", "golden", "lipschitz.json")
    try:
        with open(path) as f:
            return json.load(f)[w.key]["L"]
    except (OSError, KeyError):
        return None


def reference_solution(api, torch, g, b, w, ref_iters, alpha):
    """x* by preconditioned PDHG (the reference method of the data-splitting figure), with the
    squared relative change over its second half as a convergence check."""
    t0 = time.perf_counter()
    half = ref_iters // 2
    xs, y1, y2 = api.pdhg(g, b, alpha=alpha, n_iters=half, nonneg=w.nonneg)
    x_half = xs.clone()
    api.pdhg(g, b, alpha=alpha, n_iters=ref_iters - half, nonneg=w.nonneg, x=xs, y1=y1, y2=y2)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    xstar = xs.double()
    n2 = float((xstar * xstar).sum())
    ref_change = float(((xstar - x_half.double()) ** 2).sum()) / n2
    log(f"bench: reference x*: {ref_iters} PDHG iterations in {t_ref:.1f} s; squared change over "
        f"the last {ref_iters - half}: {ref_change:.2e}")
    return {"xstar": xstar, "n2": n2, "seconds": t_ref, "change": ref_change, "iterations": ref_iters}


def run_to_eps(torch, step, current, ref, passes):
    """Data passes (calls of `step`) until ||x - x*||^2 / ||x*||^2 < 1e-5, at most `passes`; the
    passes and seconds (GPU work of the steps only) at which 1e-3 and 1e-5 were first reached."""
    def err(x):
        d = x.double() - ref["xstar"]
        return float((d * d).sum()) / ref["n2"]
    elapsed, hit, e_now, e = 0.0, {}, None, 0
    for e in range(1, passes + 1):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t1
        e_now = err(current())
        for eps in (1e-3, 1e-5):
            if eps not in hit and e_now < eps:
                hit[eps] = (e, elapsed)
        if 1e-5 in hit:
            break
    rec = {"passes": e, "seconds": round(elapsed, 4), "final_sq_rel_err": e_now}
    for eps, tag in ((1e-3, "1e-3"), (1e-5, "1e-5")):
        rec[f"passes_to_{tag}"] = hit[eps][0] if eps in hit else None
        rec[f"seconds_to_{tag}"] = round(hit[eps][1], 4) if eps in hit else None
    return rec


def time_to_eps(api, torch, g, b, w, gamma, ref, passes, alpha):
    """The paper's protocol (Sec. 2.1): wall time and data passes until the squared relative
    error ||x - x*||^2 / ||x*||^2 falls below 1e-3 and 1e-5 (at most `passes` data passes; one
    pass = N subset gradients, or one iteration of a deterministic method), with x* from
    reference_solution.  Step sizes as in the paper's comparison of all methods (Sec. 3): 1.99/L
    for ISTA and deterministic ProxSkip, 1/L for FISTA and the SVRG family, 1/(3L) for SAGA;
    `gamma` is 1/L."""
    g1 = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=1, device=g.device)
    api.autotune(g1, reps=3, cache_path=PLANS_FILE, store=False)
    specs = [("ProxSVRGSkip p=0.1", g, dict(p=0.1)),
             ("ProxSVRGSkip p=0.02", g, dict(p=0.02)),
             ("ProxSVRG", g, dict(p=1.0, plain_prox_svrg=True)),
             ("ProxLSVRGSkip p=0.1", g, dict(p=0.1, estimator="lsvrg")),
             ("ProxLSVRG", g, dict(p=1.0, estimator="lsvrg", plain_prox_svrg=True)),
             ("ProxSAGASkip p=0.1", g, dict(p=0.1, estimator="saga", gamma=gamma / 3.0)),
             ("ProxSAGA", g, dict(p=1.0, estimator="saga", plain_prox_svrg=True, gamma=gamma / 3.0)),
             ("ISTA", g1, dict(p=1.0, plain_prox_svrg=True, gamma=1.99 * gamma)),
             ("ProxSkip p=0.1", g1, dict(p=0.1, gamma=1.99 * gamma)),
             ("FISTA", g1, None)]
    runs = []
    for label, geom, kw in specs:
        if kw is None:
            f = api.Fista(geom, b, gamma=gamma, alpha=alpha, fgp_inner=w.fgp_inner, nonneg=w.nonneg)
            step, current = (lambda: f.run(1)), (lambda: f.x)
        else:
            prm = dict(gamma=gamma, alpha=alpha, fgp_inner=w.fgp_inner, n_epochs=passes,
                       nonneg=w.nonneg, seed=w.seed + 2)
            prm.update(kw)
            sv = api.Solver(geom, b, api.SolverParams(**prm))
            step, current = (lambda: sv.epochs(1)), (lambda: sv.x)
        rec = {"method": label, **run_to_eps(torch, step, current, ref, passes)}
        runs.append(rec)
        log(f"bench: to eps {label}: " + " ".join(f"{k}={v}" for k, v in rec.items() if k != "method"))
    del g1
    # prox skipping against the non-skipped ProxSVRG at the same threshold (wall time)
    by = {r["method"]: r for r in runs}
    speedup = {}
    for tag in ("1e-3", "1e-5"):
        base = by["ProxSVRG"][f"seconds_to_{tag}"]
        for m in ("ProxSVRGSkip p=0.1", "ProxSVRGSkip p=0.02", "ProxLSVRGSkip p=0.1"):
            t = by[m][f"seconds_to_{tag}"]
            if base and t:
                speedup[f"{m} at {tag}"] = round(base / t, 2)
    return {"alpha": alpha, "skip_speedup_vs_ProxSVRG": speedup,
            "reference": {"method": "preconditioned PDHG", "iterations": ref["iterations"],
                          "seconds": round(ref["seconds"], 2), "sq_change_last_half": ref["change"]},
            "criterion": "||x - x*||^2 / ||x*||^2 < eps, at most %d data passes" % passes,
            "runs": runs}


def subset_sweep(api, torch, w, b, gamma, ref, passes, alpha, p=0.3, ns=(10, 50, 100, 200, 400)):
    """ProxSVRGSkip at p = 0.3 against the non-skipped ProxSVRG over the number of subsets N, on
    the time-to-epsilon problem (the paper varies N at fixed p in its ProxSVRG comparison, Sec.
    2.1): data passes and seconds to 1e-3 and 1e-5 of the squared relative error, at most
    `passes` passes.  Each N's geometry is tuned (plans not stored); gamma = 1/L for all N (L
    does not depend on the split)."""
    out = []
    for n in ns:
        gn = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=n)
        api.autotune(gn, reps=3, cache_path=PLANS_FILE, store=False)
        row = {"N": n}
        for label, kw in (("skip", dict(p=p)), ("noskip", dict(p=1.0, plain_prox_svrg=True))):
            sv = api.Solver(gn, b, api.SolverParams(gamma=gamma, alpha=alpha, fgp_inner=w.fgp_inner,
                                                    n_epochs=passes, nonneg=w.nonneg, seed=w.seed + 2, **kw))
            row[label] = run_to_eps(torch, lambda: sv.epochs(1), lambda: sv.x, ref, passes)
            del sv
        for tag in ("1e-3", "1e-5"):
            a, c = row["noskip"][f"seconds_to_{tag}"], row["skip"][f"seconds_to_{tag}"]
            row[f"skip_speedup_at_{tag}"] = round(a / c, 2) if a and c else None
        log(f"bench: subset sweep N={n}: {row}")
        out.append(row)
        del gn
    return {"p": p, "alpha": alpha, "criterion": "||x - x*||^2 / ||x*||^2 < eps, at most %d data passes" % passes,
            "rows": out}


def volume_ops():
    """One subset projection, one subset backprojection, a 10-iteration 3D TV prox and one
    all-angle projection and backprojection on the 256 x 1024^2 volume geometry with its stored
    plan and random inputs: a short program for hardware counters (under counter collection the
    synthetic sinogram takes minutes)."""
    import torch
    from paper_2602_09527_amd import api, workloads
    w = workloads.VOLUME_3D
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, nz=w.nz)
    plan = api.autotune(g, reps=2, cache_path=PLANS_FILE, store=False, tune_missing=False)
    log(f"bench: volume ops, launch plan {plan}")
    x = torch.rand(g.image_shape, device="cuda")
    y = torch.empty(g.sino_shape(0), device="cuda")
    api.project(g, x, 0, out=y)
    torch.cuda.synchronize()
    log("bench: volume ops: subset projection done")
    api.backproject(g, y, 0, out=x)
    torch.cuda.synchronize()
    log("bench: volume ops: subset backprojection done")
    dual = torch.zeros(g.dual_shape(), device="cuda")
    api.tv_prox(g, x, 1e-4, 10, dual=dual, out=torch.empty_like(x))
    torch.cuda.synchronize()
    log("bench: volume ops: 10-iteration prox done")
    del dual, y
    yf = torch.empty(g.sino_shape(-1), device="cuda")
    api.project(g, x, -1, out=yf)
    torch.cuda.synchronize()
    log("bench: volume ops: all-angle projection done")
    api.backproject(g, yf, -1, out=x)
    torch.cuda.synchronize()
    log("bench: volume ops: all-angle backprojection done")


def volume_leg(epochs, warmup, log_fn, graph_check=True, plan_check=True, oracle_ops=True):
    """The 256 x 1024^2 volume (1800 angles x 1448 bins, 30 subsets, 3D TV, p = 0.05): `epochs`
    timed ProxSkip-SVRG epochs after `warmup`, per-operator times with the stored plan and with
    the automatic one, one epoch eager against the same epoch issued as a captured HIP graph, and
    the FP64 oracle's per-operator times on a few slices of the same geometry, extrapolated to the
    volume (labelled as such)."""
    import numpy as np
    import torch
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.VOLUME_3D
    dev = torch.device("cuda", 0)
    t0 = time.time()
    ells = synth.random_ellipses(w.seed, 10, dims=3)
    clean = synth.analytic_sinogram_torch(ells, w.nx, w.ny, w.n_angles, w.n_bins, nz=w.nz,
                                          device=dev, dtype=torch.float32)
    b = synth.poisson_log_noise_torch(clean, w.seed + 1)
    del clean
    torch.cuda.synchronize()
    t_data = time.time() - t0
    log_fn(f"bench: volume data {tuple(b.shape)} in {t_data:.1f} s")
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, nz=w.nz, device=dev)
    plan = api.autotune(g, reps=2, cache_path=PLANS_FILE, store=False, tune_missing=False)
    L = stored_L(w) or api.lipschitz(g, 20)
    K, W = epochs, warmup
    N = w.n_subsets
    prm = dict(gamma=1.0 / L, p=w.p, alpha=w.alpha, fgp_inner=w.fgp_inner, nonneg=w.nonneg,
               seed=w.seed + 2)
    s = api.Solver(g, b, api.SolverParams(n_epochs=W + K, **prm))
    s.epochs(W)
    s.query()
    torch.cuda.synchronize()
    log_fn(f"bench: volume {W} warm-up epochs done")
    # the same state continued by a second handle, for the graph comparison below
    state = (s.x.clone(), s.h.clone(), s.dual.clone()) if graph_check else None
    per_epoch = []
    calls0 = s.query()["prox_calls"]
    t1 = time.perf_counter()
    for e in range(K):
        te = time.perf_counter()
        c0 = s.query()["prox_calls"]
        s.epochs(1)
        torch.cuda.synchronize()
        per_epoch.append((time.perf_counter() - te, s.query()["prox_calls"] - c0))
        log_fn(f"bench: volume epoch {e + 1}/{K}: {per_epoch[-1][0]:.3f} s, "
               f"{per_epoch[-1][1]} prox calls")
    el = time.perf_counter() - t1
    st = s.query()
    rec = {"workload": w.name, "volume": f"{w.nz}x{w.ny}x{w.nx}", "angles": w.n_angles,
           "bins": w.n_bins, "subsets": N, "p": w.p, "alpha": w.alpha, "fgp_inner": w.fgp_inner,
           "tv": "3D isotropic", "noise": w.noise, "data_s": round(t_data, 2),
           "epochs": K, "warmup": W, "s_per_epoch": round(el / K, 4),
           "epochs_per_s": round(K / el, 4), "prox_calls": st["prox_calls"] - calls0,
           "epoch_s_and_prox_calls": [[round(a, 4), c] for a, c in per_epoch], "plan": plan}

    def event_time(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    del s
    torch.cuda.empty_cache()

    # per-operator times: stored (tuned) plan against the automatic plan
    n = w.nx * w.ny * w.nz
    a = g.subset_size(0)
    x = torch.rand(g.image_shape, device=dev)
    ysub = torch.empty(g.sino_shape(0), device=dev)
    img = torch.empty_like(x)
    dual = torch.zeros(g.dual_shape(), device=dev)
    copy_src = torch.ones(256 * 1024 * 1024, device=dev)
    copy_dst = torch.empty_like(copy_src)
    t_copy = event_time(lambda: copy_dst.copy_(copy_src), reps=5)
    copy_gbs = 2.0 * copy_src.numel() * 4 / t_copy / 1e9
    del copy_src, copy_dst
    def ops(geom):
        tp = event_time(lambda: api.project(geom, x, 0, out=ysub))
        tb = event_time(lambda: api.backproject(geom, ysub, 0, out=img))
        # one inner iteration: a 12-iteration prox less a 2-iteration one (the finalize and the
        # copies around the iterations cancel), per iteration
        t12 = event_time(lambda: api.tv_prox(geom, x, 1e-4, 12, dual=dual, out=img), reps=2)
        t2 = event_time(lambda: api.tv_prox(geom, x, 1e-4, 2, dual=dual, out=img), reps=2)
        return tp, tb, (t12 - t2) / 10
    t_fp, t_bp, t_it = ops(g)
    steps_fp = a * w.n_bins * w.nz * max(w.nx, w.ny)
    form = g.get_plan()["fgp3d_form"]
    # bytes per voxel and iteration: 40 as one iteration per launch moves them (read v, p (3),
    # p_prev (3); write p (3)); a two-iteration launch reads 7 and writes 6 values per voxel
    b_one = 40.0 * n
    b_form = (26.0 if form >= 2 else 40.0) * n
    rec["kernels"] = {
        "project_subset_ms": round(t_fp * 1e3, 3),
        "project_subset_gsamples_per_s": round(steps_fp / t_fp / 1e9, 1),
        "backproject_subset_ms": round(t_bp * 1e3, 3),
        "fgp3d_form": form,
        "fgp3d_iteration_ms": round(t_it * 1e3, 3),
        "fgp3d_gbs_at_40B": round(b_one / t_it / 1e9, 1),
        "fgp3d_hbm_frac_at_40B": round(b_one / t_it / 1e9 / HBM_PEAK_GBS, 4),
        "fgp3d_gbs_moved": round(b_form / t_it / 1e9, 1),
        "fgp3d_hbm_frac_moved": round(b_form / t_it / 1e9 / HBM_PEAK_GBS, 4),
        "device_copy_gbs": round(copy_gbs, 1)}
    log_fn(f"bench: volume kernels {rec['kernels']}")
    if plan_check:
        gd = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=N, nz=w.nz, device=dev)
        d_fp, d_bp, d_tv = ops(gd)
        rec["tuned_vs_automatic_plan"] = {
            "automatic_plan": gd.get_plan(),
            "project_subset_ms": [round(t_fp * 1e3, 3), round(d_fp * 1e3, 3)],
            "backproject_subset_ms": [round(t_bp * 1e3, 3), round(d_bp * 1e3, 3)],
            "fgp3d_iteration_ms": [round(t_it * 1e3, 3), round(d_tv * 1e3, 3)]}
        log_fn(f"bench: volume tuned vs automatic {rec['tuned_vs_automatic_plan']}")
        del gd
    del x, ysub, img, dual
    torch.cuda.empty_cache()
    # last: kernels timed after HIP graphs have run measured slower here (3D FGP 1.9 -> 2.7 ms per
    # iteration), so the per-operator times above come first
    if graph_check:
        # epoch W + 1 eager (a fresh handle from the saved state) against the same epoch as a HIP
        # graph (another handle from the same state): identical work, bit for bit the same x
        xs_, hs_, ds_ = state
        times = {}
        xs_out = {}
        for mode in ("eager", "graph"):
            h2 = api.Solver(g, b, api.SolverParams(n_epochs=1, k0=W * N, **prm),
                            x=xs_.clone(), h=hs_.clone(), dual=ds_.clone())
            torch.cuda.synchronize()
            tg = time.perf_counter()
            h2.epochs(1, graph=(mode == "graph"))
            torch.cuda.synchronize()
            times[mode] = time.perf_counter() - tg
            xs_out[mode] = h2.x.clone()
            del h2
            log_fn(f"bench: volume epoch {W + 1} {mode}: {times[mode]:.3f} s")
        rec["graph_vs_eager"] = {"epoch": W + 1, "eager_s": round(times["eager"], 4),
                                 "graph_s": round(times["graph"], 4),
                                 "graph_over_eager": round(times["graph"] / times["eager"], 4),
                                 "bitwise_equal": bool(torch.equal(xs_out["eager"], xs_out["graph"]))}
        del xs_out, state, xs_, hs_, ds_
        torch.cuda.empty_cache()

    if oracle_ops:
        rec["oracle_ops"] = oracle_volume_ops(w, log_fn)
    return rec


def oracle_volume_ops(w, log_fn, nz_proj=2, nz_tv=4):
    """The FP64 oracle's time for one subset projection, one subset backprojection (2 slices of
    the volume's geometry) and one 3D FGP iteration (4 slices), each extrapolated to the 256
    slices, and an epoch estimated from them (labelled extrapolated)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    og = oracle.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, nz=nz_proj)
    x = rng.random((nz_proj, w.ny, w.nx))
    t = time.perf_counter()
    y = oracle.project(og, x, 0)
    t_fp = time.perf_counter() - t
    t = time.perf_counter()
    oracle.backproject(og, y, 0)
    t_bp = time.perf_counter() - t
    v = rng.random((nz_tv, w.ny, w.nx))
    dual = np.zeros((3, nz_tv, w.ny, w.nx))
    t = time.perf_counter()
    oracle.tv_prox_fgp(v, 1e-2, 1, nonneg=True, dual=dual)
    t_tv = time.perf_counter() - t
    sp, st_ = w.nz / nz_proj, w.nz / nz_tv
    fp, bp, tv = t_fp * sp, t_bp * sp, t_tv * st_
    N = w.n_subsets
    # an SVRG epoch: the snapshot's all-angle pair (N subsets' worth) plus N subset pairs, and
    # p N prox calls of fgp_inner iterations on average
    epoch = 2 * N * (fp + bp) + w.p * N * w.fgp_inner * tv
    rec = {"threads": oracle.num_threads(),
           "sample": f"subset projection and backprojection on {nz_proj} slices, one 3D FGP "
                     f"iteration on {nz_tv} slices of the 1024^2 geometry (random inputs), "
                     f"scaled to {w.nz} slices",
           "project_subset_s_extrapolated": round(fp, 3),
           "backproject_subset_s_extrapolated": round(bp, 3),
           "fgp3d_iteration_s_extrapolated": round(tv, 3),
           "epoch_s_extrapolated": round(epoch, 1),
           "epochs_per_s_extrapolated": round(1.0 / epoch, 6)}
    log_fn(f"bench: volume oracle ops {rec}")
    return rec


def bench_volume(args):
    """--volume: the 256 x 1024^2 volume alone, one JSON line with its epochs per second."""
    rec = volume_leg(args.steps, args.warmup, log)
    out = {"metric": METRIC, "value": rec["epochs_per_s"], "unit": "epochs/s", "n_gpus": 1,
           "steps": rec["epochs"], "warmup": rec["warmup"], "ms_per_step": round(1e3 * rec["s_per_epoch"], 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": rec["workload"]}, "volume": rec}
    print(json.dumps(out), flush=True)


def bench_batch(dev, log_fn, n_slices=64, epochs=10):
    """Epochs per second of 64 independent 128^2 solves batched in lockstep, against the same
    solves run one after another."""
    import torch
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.SMALL_2D
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, device=dev)
    L = stored_L(w) or api.lipschitz(g, 50)
    api.autotune(g, reps=5, cache_path=PLANS_FILE, store=False)
    bs = []
    for j in range(n_slices):
        prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed + 10 * j,
                                  noise=w.noise, with_phantom=False)
        bs.append(torch.from_numpy(prob.b).to(device=dev, dtype=torch.float32))

    def solvers():
        return [api.Solver(g, b, api.SolverParams(gamma=1.0 / L, p=w.p, alpha=w.alpha,
                                                  fgp_inner=w.fgp_inner, n_epochs=epochs + 1,
                                                  nonneg=w.nonneg, seed=w.seed + 2 + 10 * j))
                for j, b in enumerate(bs)]
    sv = solvers()
    api.run_epochs(sv, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    api.run_epochs(sv, epochs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    sq = solvers()
    for s in sq:
        s.epochs(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sq:
        s.epochs(epochs)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    same = all(torch.equal(a.x, b.x) for a, b in zip(sv, sq))
    rec = {"workload": f"{n_slices} x {w.name}", "epochs": epochs,
           "batched_slice_epochs_per_s": round(n_slices * epochs / t_batch, 1),
           "sequential_slice_epochs_per_s": round(n_slices * epochs / t_seq, 1),
           "speedup": round(t_seq / t_batch, 3), "bitwise_equal_to_sequential": bool(same)}
    log_fn(f"bench: batch {rec}")
    return rec


def bench_serve(args, dev, log_fn):
    """A Poisson trace of mixed-size reconstructions, each solved to 1e-4 relative change (or
    the epoch cap), served with continuous batching, against the same trace served one request
    at a time."""
    from paper_2602_09527_amd import serve
    trace = serve.make_trace(args.serve_requests, args.serve_rate, seed=505)
    geoms = serve.GeometryCache(dev, power_iters=30)
    geoms.warm(trace)
    bank = serve.data_bank(trace, dev)
    cfg = serve.ServeConfig(max_epochs=args.serve_cap)
    res, wall = serve.serve(trace, cfg, bank, geoms)
    batched = serve.summarize(res, wall)
    log_fn(f"bench: serving (batched) {batched}")
    res2, wall2 = serve.serve_sequential(trace, cfg, bank, geoms)
    seq = serve.summarize(res2, wall2)
    log_fn(f"bench: serving (one at a time) {seq}")
    rel = [r["last_rel_change"] for r in res]
    return {"trace": f"{args.serve_requests} requests, Poisson {args.serve_rate}/s, sides "
                     f"{{128..1024}}, angles {{90..1800}}, bins 1.5 N, p = {cfg.p}, "
                     f"alpha = {cfg.alpha}, {cfg.fgp_inner} FGP iterations, stop at relative "
                     f"change < {cfg.tol} or {cfg.max_epochs} epochs",
            "continuous_batching": batched, "one_at_a_time": seq,
            "converged": batched["converged"],
            "relative_change_at_stop": {"min": min(rel), "median": float(sorted(rel)[len(rel) // 2]),
                                        "max": max(rel)},
            "arrival_span_s": round(trace[-1].arrival, 3),
            # when the arrivals outpace the service (the last result comes well after the last
            # arrival) the GPU is busy from the first arrival to the last result, and the
            # measured throughput is the highest rate this mix can be sustained at
            "sustainable_req_per_s": ({"continuous_batching": batched["throughput_req_s"],
                                       "one_at_a_time": seq["throughput_req_s"]}
                                      if min(wall, wall2) > 1.5 * trace[-1].arrival else None)}


def calibrate_copy():
    import torch
    n = 64 * 1024 * 1024  # 256 MiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_each_way": 4 * n, "launches": 3}), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_one_thread(og, b, kw, threads, epochs=1):
    """The same oracle solve on one thread (results do not depend on the thread count)."""
    import oracle
    oracle.set_num_threads(1)
    try:
        t = time.perf_counter()
        oracle.proxskip_svrg(og, b, **{**kw, "n_epochs": epochs})
        el = time.perf_counter() - t
    finally:
        oracle.set_num_threads(threads)
    log(f"bench: oracle on 1 thread: {epochs} epoch(s) in {el:.1f} s")
    return {"epochs": epochs, "epochs_per_s": round(epochs / el, 4), "seconds": round(el, 2)}


def oracle_other_configs(threads):
    """The oracle on the other fixed workloads: the full 30-epoch 128^2 solve, and the forward and
    backward projection of two images of the 64-image autograd batch (extrapolated to 64)."""
    import numpy as np
    import oracle
    from paper_2602_09527_amd import synth, workloads
    out = {"threads": threads}
    w = workloads.SMALL_2D
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed, noise=w.noise,
                              with_phantom=False)
    og = oracle.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
    t = time.perf_counter()
    _, _, _, st, _ = oracle.proxskip_svrg(og, prob.b, gamma=1.0 / stored_L(w), p=w.p, alpha=w.alpha,
                                          fgp_inner=w.fgp_inner, n_epochs=w.n_epochs,
                                          nonneg=w.nonneg, seed=w.seed + 2)
    el = time.perf_counter() - t
    out[w.name] = {"epochs": w.n_epochs, "seconds": round(el, 2),
                   "epochs_per_s": round(w.n_epochs / el, 3), "prox_calls": st["prox_calls"]}
    wa = workloads.AUTOGRAD_BATCH
    two = 2
    oa = oracle.Geometry(wa.nx, wa.ny, wa.n_angles, wa.n_bins, nz=two)
    xa = np.random.default_rng(0).random((two, wa.ny, wa.nx))
    t = time.perf_counter()
    ya = oracle.project(oa, xa, -1)
    tf = time.perf_counter() - t
    t = time.perf_counter()
    oracle.backproject(oa, ya, -1)
    tb = time.perf_counter() - t
    out[wa.name] = {"sample": f"{two} images, extrapolated to {wa.nz}",
                    "forward_images_per_s": round(two / tf, 2),
                    "backward_images_per_s": round(two / tb, 2),
                    "forward_s_per_batch_extrapolated": round(tf * wa.nz / two, 2),
                    "backward_s_per_batch_extrapolated": round(tb * wa.nz / two, 2)}
    log(f"bench: oracle on the other workloads {out}")
    return out


def solve_only(args):
    """--solve WORKLOAD: the workload's ProxSkip-SVRG solve alone, --steps timed epochs after
    --warmup, on its stored plan and stored step size (a short program for kernel traces)."""
    import torch
    from paper_2602_09527_amd import api, synth, workloads
    w = workloads.ALL[args.solve]
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed, noise=w.noise,
                              with_phantom=False)
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
    plan = api.autotune(g, reps=3, cache_path=PLANS_FILE, store=False)
    b = torch.from_numpy(prob.b).to(device="cuda", dtype=torch.float32)
    s = api.Solver(g, b, api.SolverParams(gamma=1.0 / stored_L(w), p=w.p, alpha=w.alpha,
                                          fgp_inner=w.fgp_inner, n_epochs=args.warmup + args.steps,
                                          nonneg=w.nonneg, seed=w.seed + 2))
    s.epochs(args.warmup)
    s.query()
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.epochs(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    st = s.query()
    print(json.dumps({"workload": w.name, "epochs": args.steps, "epochs_per_s": round(args.steps / el, 2),
                      "prox_calls": st["prox_calls"], "plan": plan}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the solve runs on one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.volume_ops:
        volume_ops()
        return
    if args.volume:
        bench_volume(args)
        return
    if args.solve:
        solve_only(args)
        return
    from paper_2602_09527_amd import api, synth, workloads

    w = workloads.SINGLE_2D
    p = w.p if args.p is None else args.p
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"bench: workload {w.name}: {w.nx}x{w.ny}, {w.n_angles} angles x {w.n_bins} bins, "
        f"N={w.n_subsets}, p={p}, alpha={w.alpha}, fgp_inner={w.fgp_inner}")
    t0 = time.time()
    prob = synth.make_problem(w.nx, w.ny, w.n_angles, w.n_bins, seed=w.seed, noise=w.noise,
                              with_phantom=False)
    log(f"bench: synthetic data in {time.time() - t0:.1f} s")
    g = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets, device=dev)
    b = torch.from_numpy(prob.b).to(device=dev, dtype=torch.float32)
    # gamma = 1/L with L from the oracle's FP64 power method, stored with the tests: the timed
    # solve and its oracle parity check below use the identical double
    L = stored_L(w)
    if L is None:
        L = api.lipschitz(g, 50)
        log(f"bench: no stored L for {w.key}; GPU power method L = {L:.6f}")
    gamma = 1.0 / L
    log(f"bench: L = {L:.9f} (stored, oracle power method)")
    plan = api.autotune(g, reps=5, cache_path=PLANS_FILE, store=False)
    log(f"bench: launch plan {plan}")

    def params(n_epochs, **kw):
        d = dict(gamma=gamma, p=p, alpha=w.alpha, fgp_inner=w.fgp_inner, n_epochs=n_epochs,
                 nonneg=w.nonneg, seed=w.seed + 2)
        d.update(kw)
        return api.SolverParams(**d)

    # ---- timed region: K epochs of one continuing solve ------------------------------------
    K, W = args.steps, args.warmup
    s = api.Solver(g, b, params(W + K))
    s.epochs(W)
    s.query()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.epochs(K)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = s.query()
    eps = K / el
    log(f"bench: {K} epochs in {el:.4f} s -> {eps:.1f} epochs/s; prox calls {st['prox_calls']}, "
        f"last rel change {st['last_rel_change']:.3e}")

    # ---- dominant kernels: HIP events around their launches on the current stream ---------
    def event_time(fn, reps=30):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3  # seconds per launch

    x = s.x
    ysub = torch.empty(g.sino_shape(0), dtype=torch.float32, device=dev)
    yfull = torch.empty(g.sino_shape(-1), dtype=torch.float32, device=dev)
    img = torch.empty_like(x)
    t_bp_full = event_time(lambda: api.backproject(g, yfull, -1, out=img))
    t_bp_sub = event_time(lambda: api.backproject(g, ysub, 0, out=img))
    t_fp_full = event_time(lambda: api.project(g, x, -1, out=yfull))
    t_fp_sub = event_time(lambda: api.project(g, x, 0, out=ysub))
    n = w.nx * w.ny
    a_sub = g.subset_size(0)
    samples_full = w.n_angles * w.n_bins * max(w.nx, w.ny)   # ray-row crossings, all angles
    samples_sub = a_sub * w.n_bins * max(w.nx, w.ny)
    bytes_fp_full = 4.0 * (n + w.n_angles * w.n_bins)
    bytes_fp_sub = 4.0 * (2 * n + a_sub * w.n_bins)
    bytes_bp_full = 4.0 * (w.n_angles * w.n_bins + n)

    def krec(t, samples, ops, nbytes):
        return {"us": round(t * 1e6, 2), "gsamples_per_s": round(samples / t / 1e9, 1),
                "alu_tops": round(ops * samples / t / 1e12, 3),
                "alu_frac": round(ops * samples / t / 1e12 / ALU_PEAK_TOPS, 4),
                "algorithmic_gbs": round(nbytes / t / 1e9, 2)}
    kern = {
        "backproject_full": krec(t_bp_full, samples_full, OPS_BACKPROJECT, bytes_bp_full),
        "project_full": krec(t_fp_full, samples_full, OPS_PROJECT, bytes_fp_full),
        "backproject_subset": krec(t_bp_sub, samples_sub, OPS_BACKPROJECT, 4.0 * (a_sub * w.n_bins + n)),
        "project_subset": krec(t_fp_sub, samples_sub, OPS_PROJECT, bytes_fp_sub),
    }
    for k_, v in kern.items():
        log(f"bench: {k_}: " + " ".join(f"{kk}={vv}" for kk, vv in v.items()))
    # ---- per-kernel GPU time inside the solve: the library's HIP events around every launch of
    # each class over E_t more epochs (a second pass: the events would perturb the timed one) ---
    E_t = 20
    s2 = api.Solver(g, b, params(W + E_t))
    s2.epochs(W)
    s2.query()
    torch.cuda.synchronize()
    classes = ("backproject_subset", "project_subset", "backproject_full", "project_full",
               "backproject_combine", "project_reduce", "backproject_gather", "fgp2d")
    with api.KernelTimer(classes) as kt:
        t1 = time.perf_counter()
        s2.epochs(E_t)
        torch.cuda.synchronize()
        el_t = time.perf_counter() - t1
        per = {c: kt.result(c) for c in classes}
    del s2
    # algorithmic work per launch: lane operations of the ray steps for the projector and the
    # backprojector (SURVEY's per-sample figures), none counted for the other classes
    samples = {"backproject_subset": samples_sub, "project_subset": samples_sub,
               "backproject_full": samples_full, "project_full": samples_full}
    ops = {"backproject_subset": OPS_BACKPROJECT, "project_subset": OPS_PROJECT,
           "backproject_full": OPS_BACKPROJECT, "project_full": OPS_PROJECT}
    breakdown = {}
    for c, (ms, nl) in per.items():
        if nl == 0:
            continue
        r = {"launches_per_epoch": round(nl / E_t, 2), "us_per_launch": round(1e3 * ms / nl, 2),
             "ms_per_epoch": round(ms / E_t, 4), "share_of_epoch": round(ms / (1e3 * el_t), 4)}
        if c in samples:
            r["alu_frac"] = round(ops[c] * samples[c] / (ms / nl * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4)
        breakdown[c] = r
    log(f"bench: kernel time per epoch (library events, {E_t} epochs): {breakdown}")
    # the dominant kernel: the class with the most GPU time per epoch, then its launch timed
    # alone (library HIP events around back-to-back launches, dispatch overlapped as in the
    # solve: the in-solve events above also count each launch's dispatch)
    dom = max(breakdown, key=lambda c: breakdown[c]["ms_per_epoch"])
    alone = {c: api.kernel_time(g, c, reps=200) for c in samples}
    for c, us in alone.items():
        if c in breakdown:
            breakdown[c]["us_per_launch_alone"] = round(us, 2)
            breakdown[c]["alu_frac_alone"] = round(ops[c] * samples[c] / (us * 1e-6) / 1e12 / ALU_PEAK_TOPS, 4)
    log(f"bench: kernels alone (us per launch): {alone}")
    t_dom = (alone[dom] if dom in alone else breakdown[dom]["us_per_launch"]) * 1e-6
    names = {"backproject_subset": "k_backproject (scatter), one subset: 36 angles x 768 bins "
                                   "over 512 rows",
             "project_subset": "k_project, one subset: 36 angles x 768 bins over 512 rows",
             "backproject_full": "k_backproject (scatter), all 720 angles x 768 bins over 512 rows",
             "project_full": "k_project, all 720 angles x 768 bins over 512 rows"}
    if dom in samples:
        achieved = ops[dom] * samples[dom] / t_dom / 1e12
        traffic = measured_traffic(dom)
        roofline = {"kernel": names[dom], "bound": "alu", "achieved": round(achieved, 3),
                    "peak": round(ALU_PEAK_TOPS, 2), "unit": "Tops/s",
                    "frac": round(achieved / ALU_PEAK_TOPS, 4),
                    "traffic": round(traffic) if traffic else None,
                    "us_per_launch": round(t_dom * 1e6, 2), "ops_per_sample": ops[dom],
                    "samples_per_launch": samples[dom], "launches_per_epoch":
                    breakdown[dom]["launches_per_epoch"],
                    "timing": "HIP events around 200 back-to-back launches of the kernel alone "
                              "(kernel_time), median of three rounds; chosen as the kernel with "
                              "the most GPU time per epoch inside the solve (HIP events around "
                              "each launch over %d epochs)" % E_t}
    else:
        roofline = {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None,
                    "frac": None, "traffic": None}
    # the whole epoch: projector and backprojector lane operations over the epoch's wall time
    n_sub_iters = w.n_subsets - 1
    epoch_ops = (OPS_PROJECT + OPS_BACKPROJECT) * (n_sub_iters * samples_sub + samples_full)

    out = {
        "metric": METRIC, "value": round(eps, 3), "unit": "epochs/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(1e3 * el / K, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "image": f"{w.nx}x{w.ny}", "angles": w.n_angles,
                   "bins": w.n_bins, "subsets": w.n_subsets, "p": p, "alpha": w.alpha,
                   "fgp_inner": w.fgp_inner, "method": "ProxSkip-SVRG"},
        "roofline": roofline,
        "epoch_alu_frac": {"value": round(epoch_ops / (el / K) / 1e12 / ALU_PEAK_TOPS, 4),
                           "what": "lane operations of the projector and backprojector ray steps "
                                   "in one epoch (19 subset pairs and the snapshot's all-angle "
                                   "pair) over the epoch's wall time, against the VALU peak"},
        "kernel_time_per_epoch": breakdown,
        "plan": plan,
        "projector_hbm_gbs": kern["project_full"]["algorithmic_gbs"],
        "kernels": kern,
    }

    # ---- differentiable projector on a batch of 64 images of 256^2 (360 x 384, all angles) ---
    wa = workloads.AUTOGRAD_BATCH
    ga = api.Geometry(wa.nx, wa.ny, wa.n_angles, wa.n_bins, nz=wa.nz, device=dev)
    api.autotune(ga, cache_path=PLANS_FILE, store=False, tune_missing=False)   # its stored plan
    xa = torch.rand(ga.image_shape, device=dev)
    ya = torch.empty(ga.sino_shape(-1), device=dev)
    # the median of three rounds of 10 calls, after the warm-up call: the first round of a fresh
    # geometry's buffers ran up to 13% slower than later ones
    ta_f = sorted(event_time(lambda: api.project(ga, xa, -1, out=ya), reps=10) for _ in range(3))[1]
    ta_b = sorted(event_time(lambda: api.backproject(ga, ya, -1, out=xa), reps=10) for _ in range(3))[1]
    out["autograd_batch"] = {"workload": wa.name, "forward_images_per_s": round(wa.nz / ta_f, 1),
                             "backward_images_per_s": round(wa.nz / ta_b, 1),
                             "forward_ms": round(ta_f * 1e3, 3), "backward_ms": round(ta_b * 1e3, 3)}
    log(f"bench: autograd batch: fwd {ta_f * 1e3:.2f} ms, bwd {ta_b * 1e3:.2f} ms per 64 images")

    # ---- p sweep (same data), short runs ---------------------------------------------------
    if not args.no_sweep:
        sweep = []
        for label, kw in (("p=1", dict(p=1.0)), ("p=0.1", dict(p=0.1)), ("p=0.02", dict(p=0.02)),
                          ("ProxSVRG", dict(p=1.0, plain_prox_svrg=True)),
                          ("ProxLSVRGSkip p=0.1", dict(p=0.1, estimator="lsvrg")),
                          ("ProxSAGASkip p=0.1", dict(p=0.1, estimator="saga", gamma=gamma / 3.0))):
            E = 20
            sv = api.Solver(g, b, params(E + 2, **kw))
            sv.epochs(2)
            sv.query()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sv.epochs(E)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            q = sv.query()
            sweep.append({"run": label, "epochs_per_s": round(E / dt, 2),
                          "prox_calls": q["prox_calls"], "rel_change": q["last_rel_change"]})
            log(f"bench: sweep {label}: {E / dt:.1f} epochs/s, prox calls {q['prox_calls']}")
        # deterministic methods (one data pass per iteration): ISTA and ProxSkip as Algorithm 1
        # with one subset, and FISTA
        g1 = api.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=1, device=dev)
        api.autotune(g1, reps=3, cache_path=PLANS_FILE, store=False)
        for label, kw in (("ISTA", dict(p=1.0, plain_prox_svrg=True)), ("ProxSkip p=0.1", dict(p=0.1))):
            E = 10
            sv = api.Solver(g1, b, params(E + 2, **kw))
            sv.epochs(2)
            sv.query()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sv.epochs(E)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            q = sv.query()
            sweep.append({"run": label, "epochs_per_s": round(E / dt, 2),
                          "prox_calls": q["prox_calls"], "rel_change": q["last_rel_change"]})
            log(f"bench: sweep {label}: {E / dt:.1f} iterations/s, prox calls {q['prox_calls']}")
        E = 10
        fs = api.Fista(g1, b, gamma=gamma, alpha=w.alpha, fgp_inner=w.fgp_inner).run(2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fs.run(E)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        sweep.append({"run": "FISTA", "epochs_per_s": round(E / dt, 2), "prox_calls": E,
                      "rel_change": None})
        log(f"bench: sweep FISTA: {E / dt:.1f} iterations/s")
        del g1
        out["sweep"] = sweep

    # ---- time to epsilon against the reference x* ------------------------------------------
    if not args.no_eps or args.subset_sweep:
        ref = reference_solution(api, torch, g, b, w, args.ref_iters, args.eps_alpha)
        if not args.no_eps:
            out["time_to_eps"] = time_to_eps(api, torch, g, b, w, gamma, ref, args.eps_passes, args.eps_alpha)
        if args.subset_sweep:
            out["subset_sweep"] = subset_sweep(api, torch, w, b, gamma, ref, args.eps_passes, args.eps_alpha)
        del ref

    # ---- batched independent slices: 64 solves of 128^2 (180 x 128, N = 10) ----------------
    if not args.no_batch:
        out["batch"] = bench_batch(dev, log)

    # ---- serving: Poisson trace of mixed sizes, continuous batching vs one at a time ---------
    if not args.no_serve:
        out["serving"] = bench_serve(args, dev, log)

    # ---- the 256 x 1024^2 volume: a bounded leg (1 warm-up + 2 timed epochs by default) ------
    vol = None
    if not args.no_volume:
        torch.cuda.empty_cache()
        vol = volume_leg(args.volume_epochs, 1, log, oracle_ops=not args.no_cpu_baseline)
        torch.cuda.empty_cache()

    # ---- CPU oracle baseline on a bounded sample + parity of that sample -------------------
    if not args.no_cpu_baseline:
        import oracle
        E = args.cpu_epochs
        og = oracle.Geometry(w.nx, w.ny, w.n_angles, w.n_bins, n_subsets=w.n_subsets)
        # step size from the oracle's own power method (stored by tests/golden/make_lipschitz.py),
        # the same double on both sides of the parity check
        with open(os.path.join(ROOT, "tests", "golden", "lipschitz.json")) as f:
            gamma_o = 1.0 / json.load(f)[w.key]["L"]
        kw = dict(gamma=gamma_o, p=p, alpha=w.alpha, fgp_inner=w.fgp_inner, n_epochs=E,
                  nonneg=w.nonneg, seed=w.seed + 2)
        t1 = time.perf_counter()
        c0 = time.process_time()
        xo, _, _, so, _ = oracle.proxskip_svrg(og, prob.b, **kw)
        cpu_wall = time.perf_counter() - t1
        cpu_proc = time.process_time() - c0
        threads = oracle.num_threads()
        xg, _, _, sg = api.solve(g, b, api.SolverParams(**kw))
        torch.cuda.synchronize()
        xg = xg.cpu().numpy().astype(np.float64)
        rel = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
        out["cpu_baseline"] = {"value": round(E / cpu_wall, 4), "unit": "epochs/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{E} epochs of the same solve from x0 = 0 "
                                         f"(FP64, OpenMP over output elements); "
                                         f"{cpu_wall:.1f} s wall, {cpu_proc:.1f} s CPU",
                               "cpu_model": cpu_model()}
        out["parity"] = {"epochs": E, "rel_l2_vs_oracle": rel, "bar": 1e-4,
                         "prox_calls_gpu": sg["prox_calls"], "prox_calls_oracle": so["prox_calls"],
                         "gamma_same_as_timed_solve": gamma_o == gamma}
        log(f"bench: oracle {E} epochs in {cpu_wall:.1f} s ({threads} threads); "
            f"GPU vs oracle rel L2 = {rel:.3e}")
        if not args.no_oracle_extra:
            out["cpu_baseline"]["one_thread"] = oracle_one_thread(og, prob.b, kw, threads)
            out["oracle_timings"] = oracle_other_configs(threads)
    if vol is not None:
        out["volume"] = vol
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
