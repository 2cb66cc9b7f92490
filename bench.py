#!/usr/bin/env python3
"""Benchmark of the split CHNS time step on one MI355X.

Workload: the 2D rising bubble, 256 x 512 cells on the non-dimensional box
[0,2] x [0,4], periodic sides, no-slip top / bottom, density ratio 1000,
viscosity ratio 100, Eo = We = 10, Ar = Re = 35, Fr = 1, Cn = 1.5 h, FP64.
A step is one full pass S1..S9 (CH solve, momentum predictor, pressure
projection).  Inputs are synthetic (seeded tanh bubble, fluid at rest) and
already resident in device memory when the timed region starts.

Prints one JSON line:
  value         grid cell-updates/s = cells * steps / wall-time of the timed
                region (host-side clock after a device synchronisation on
                both sides; hipEvents on the library stream agree)
  roofline      the kernel class with the largest share of device time in a
                separate instrumented pass (hipEvent pair around every launch
                on the library stream): algorithmic bytes / kernel time vs
                the 8 TB/s HBM peak
  cpu_baseline  the CPU oracle (numpy / scipy, FP64, one thread) on a bounded
                sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid cell-updates/s per time step (FP64 vs FP32+refine), %HBM roofline, adjoint/fwd"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    return ap.parse_args()


def cpu_baseline(prob, steps):
    """Oracle on the host: `steps` steps of the same workload, one thread."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import MACGrid, Params, step as ostep

    g = MACGrid(prob.n, prob.h, prob.periodic)
    prm = Params.from_props(prob.props)
    st = W.initial_state(prob)
    with threadpool_limits(limits=1):
        st = ostep(g, st, prm)          # warm-up step (not timed)
        t0 = time.perf_counter()
        for _ in range(steps):
            st = ostep(g, st, prm)
        dt = time.perf_counter() - t0
    return {"value": prob.cells * steps / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the %dx%d rising bubble after one warm-up step (%.1f s)"
                      % (steps, prob.n[0], prob.n[1], dt)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2009_06628_amd as P
    import workloads as W

    prob = W.rising_bubble(256, steps=2000)
    g = P.grid_for_problem(prob, device="cuda:0")
    st = g.new_state(W.initial_state(prob))
    stream = g.stream

    if args.warmup:
        g.step(st, args.warmup, stats=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(st, args.steps, stats=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_s = e0.elapsed_time(e1) / 1e3
    value = prob.cells * args.steps / wall
    stats = g.step(st, 1)     # one more step, outside the timed region: solver stats + diagnostics

    roof = None
    kernels = None
    if not args.no_profile and args.profile_steps > 0:
        g.set_timing(True)
        g.step(st, args.profile_steps, stats=False)
        torch.cuda.synchronize()
        kernels = g.get_timing()
        g.set_timing(False)
        dom = max(kernels, key=lambda r: r["ms"])
        achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": dom["name"], "avg_us": round(dom["ms"] * 1e3 / dom["launches"], 3),
                "bytes_per_launch": round(dom["bytes"] / dom["launches"], 1),
                "launches_per_step": round(dom["launches"] / args.profile_steps, 1),
                "share_of_kernel_time": round(dom["ms"] / sum(k["ms"] for k in kernels), 4)}

    cpu = None
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        cpu = cpu_baseline(prob, args.cpu_steps)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rising_bubble_256x512_fp64", "grid": list(prob.n), "cells": prob.cells,
                   "bc": list(prob.bc), "density_ratio": 1000, "viscosity_ratio": 100, "We": prob.props.We,
                   "Re": prob.props.Re, "dt": prob.props.dt, "event_seconds": round(ev_s, 4),
                   "iters_last_step": {"ch": stats["iters_ch"], "mom": stats["iters_mom"], "p": stats["iters_p"]},
                   "mass_minus": stats["mass_minus"], "energy": stats["energy"]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if kernels is not None:
        out["kernels"] = [{"name": k["name"], "launches": k["launches"], "ms": round(k["ms"], 3),
                           "GBs": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 1)} for k in
                          sorted(kernels, key=lambda r: -r["ms"])]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
