"""Tune the launch plans of the benchmarked and served geometries on this GPU and store them.

    python -m paper_2602_09527_amd.tune_plans [--out PATH] [--reps R] [--only SUBSTRING ...]

Writes a JSON object keyed by Geometry.key (default: plans_mi355x.json beside this file), which
bench.py and the serving loop load instead of re-tuning, so that every run -- including the ones
taken under a profiler, whose per-launch overhead would skew a fresh tuning -- uses the same
plans.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "plans_mi355x.json")


def shapes():
    from . import workloads as w
    out = []
    for wl in (w.SINGLE_2D, w.SMALL_2D, w.AUTOGRAD_BATCH, w.VOLUME_3D_REDUCED, w.VOLUME_3D):
        out.append(dict(nx=wl.nx, ny=wl.ny, nz=wl.nz, n_angles=wl.n_angles, n_bins=wl.n_bins,
                        n_subsets=wl.n_subsets))
    for side in w.SERVE_SIDES:
        for A in w.SERVE_ANGLES:
            out.append(dict(nx=side, ny=side, nz=1, n_angles=A, n_bins=3 * side // 2,
                            n_subsets=w.SERVE_SUBSETS[A]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--only", nargs="*", default=None,
                    help="re-tune only the geometries whose key contains one of these strings and "
                         "keep the other stored plans")
    args = ap.parse_args(argv)
    import torch  # noqa: F401
    from . import api
    plans = {}
    if args.only is not None and os.path.exists(args.out):
        with open(args.out) as f:
            plans = json.load(f)
    done = set()
    for s in shapes():
        g = api.Geometry(s["nx"], s["ny"], s["n_angles"], s["n_bins"], n_subsets=s["n_subsets"],
                         nz=s["nz"])
        skip = g.key in done or (args.only is not None and not any(o in g.key for o in args.only))
        if skip:   # a served shape equal to a workload's is tuned once; --only skips the rest
            del g
            continue
        done.add(g.key)
        t0 = time.perf_counter()
        reps = args.reps if s["nz"] <= 64 else max(2, args.reps // 4)   # volumes: long launches
        plans[g.key] = api.autotune(g, reps=reps, store=False)
        print(f"tune_plans: {g.key}: {plans[g.key]} ({time.perf_counter() - t0:.2f} s)", flush=True)
        del g
    with open(args.out, "w") as f:
        json.dump(plans, f, indent=1, sort_keys=True)
    print(f"tune_plans: wrote {len(plans)} plans to {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
