#!/usr/bin/env python3
"""Benchmark of the split CHNS time step on one MI355X.

Workload: the 2D rising bubble, 256 x 512 cells on the non-dimensional box
[0,2] x [0,4], periodic sides, no-slip top / bottom, density ratio 1000,
viscosity ratio 100, Eo = We = 10, Ar = Re = 35, Fr = 1, Cn = 1.5 h, FP64.
A step is one full pass S1..S9 (CH solve, momentum predictor, pressure
projection).  Inputs are synthetic (seeded tanh bubble, fluid at rest) and
already resident in device memory when the timed region starts.

Secondary measurements (key "secondary", each on its own workload, skipped
with --no-extras):
  precision_form  3D periodic drops (128^3, 16 drops, ratios 100): FP64 vs
                  FP32 multigrid under FP64 refinement, throughput ratio and
                  the state difference after the timed steps
  batched         ensemble of 512 oscillating drops (64^2 .. 256^2), FP32 +
                  refinement, autotuned form and launch shape; eager steps and
                  hipGraph-captured steps
  adjoint         oscillating drop 128^2, FP64: backward (checkpoint every 20
                  steps, segment recompute, adjoint steps) vs forward time

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
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--extras", default="precision_form,batched,adjoint",
                    help="comma-separated secondary measurements to run (subset of the default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for the HBM byte counters)")
    return ap.parse_args()


def recorded_traffic(kernel_class):
    """HBM bytes per launch of a kernel class (dispatch-weighted over its
    kernels) from the committed counter record (two rocprofv3 --pmc passes,
    FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size); None if
    the record holds no such class or the kernels' sources changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])).hexdigest()
        if h != rec["sources_sha256"]:
            return None
        for r in rec["records"]:
            if r["kernel_class"] == kernel_class:
                return r["traffic_bytes_per_launch"]
        return None
    except (OSError, ValueError, KeyError):
        return None


def _sync():
    import torch
    torch.cuda.synchronize()


def bench_precision_form(P, W, steps):
    """3D drops: FP64 vs FP32+refinement on the same input."""
    import torch
    prob = W.drops3d(128, steps=steps, **W.PRECISION_FORM_TOLERANCES)
    init = W.initial_state(prob)
    out = {"workload": "drops3d_128^3", "cells": prob.cells, "steps": steps}
    states = {}
    for name, prec in (("fp64", P.CHNS_FP64), ("fp32_refine", P.CHNS_FP32_REFINE)):
        g = P.grid_for_problem(prob, prec, device="cuda:0")
        st = g.new_state(init)
        g.step(st, 2, stats=False)
        _sync()
        t0 = time.perf_counter()
        g.step(st, steps, stats=False)
        _sync()
        dt = time.perf_counter() - t0
        out[name] = {"value": round(prob.cells * steps / dt, 1), "ms_per_step": round(dt / steps * 1e3, 3)}
        states[name] = st
        del g
    out["speedup"] = round(out["fp32_refine"]["value"] / out["fp64"]["value"], 3)
    a, b = states["fp32_refine"], states["fp64"]
    err = float((a["phi"] - b["phi"]).abs().max() / b["phi"].abs().max())
    for d in range(3):
        err = max(err, float((a["u"][d] - b["u"][d]).abs().max() / b["u"][d].abs().max().clamp_min(1e-300)))
    out["max_rel_diff_vs_fp64"] = err
    out["tolerances"] = W.PRECISION_FORM_TOLERANCES
    return out


def bench_batched(P, W, steps):
    """Batched ensemble: 512 problems, FP32 + refinement; autotuned form and
    launch shape; timed eagerly (solves run to convergence with host checks)
    and as a captured hipGraph (fixed per-solve iteration budgets)."""
    probs = W.ensemble(count=512, seed=4, steps=200, **W.PRECISION_FORM_TOLERANCES)
    b = P.create_batch(probs, P.CHNS_FP32_REFINE, device="cuda:0")
    st = b.new_state([W.initial_state(p) for p in probs])
    tune = b.autotune(st, 1)
    out = {"workload": "ensemble_512_oscillating_drops_fp32_refine", "problems": len(probs),
           "cells": b.total_cells, "steps": steps,
           "form": tune["mode"], "tile_cells": tune["tile_cells"], "graph_budgets": list(tune["budgets"]),
           "autotune_ms_per_step": {"%s_%d_%d" % (c[0], c[1], c[2]): round(c[3], 2) for c in tune["candidates"]}}
    for label, graph in (("eager", False), ("graph", True)):
        b.step(st, steps, use_graph=graph, stats=False)     # warm-up (and capture)
        _sync()
        t0 = time.perf_counter()
        stats = b.step(st, steps, use_graph=graph, stats=True)
        dt = time.perf_counter() - t0
        tot = sum(s["total_iters"] for s in stats)
        out[label] = {"value": round(b.total_cells * steps / dt, 1), "ms_per_step": round(dt / steps * 1e3, 3),
                      "pcg_iterations_per_problem_step": round(tot / (len(probs) * steps), 2),
                      "unconverged": sum(1 for s in stats if s["flags"])}
    out["value"] = out["graph"]["value"]
    out["ms_per_step"] = out["graph"]["ms_per_step"]
    return out


def bench_adjoint(P, W):
    """Oscillating drop 128^2: 40 forward steps vs the checkpointed backward."""
    import torch
    from paper_2009_06628_amd.adjoint import rollout
    steps = 40
    prob = W.adjoint_drop(128, steps=steps)
    init = W.initial_state(prob)
    g = P.create_grid(prob.n, prob.h, prob.bc, device="cuda:0")
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda:0")
    u0 = [dev(x) for x in init["u"]]
    with torch.no_grad():
        target = rollout(g, prob.props, dev(init["phi"]), u0, 1.0, 1e-3, steps)[0].clone()
    # three forward + backward passes; the first one also attaches the adjoint
    # workspace and allocates the segment records; the minimum of each is
    # reported
    fwd_s, bwd_s = [], []
    for _ in range(3):
        phi0 = dev(init["phi"]).requires_grad_(True)
        sigma = torch.tensor(1.1, dtype=torch.float64, requires_grad=True)
        mob = torch.tensor(1.2e-3, dtype=torch.float64, requires_grad=True)
        _sync()
        t0 = time.perf_counter()
        out = rollout(g, prob.props, phi0, u0, sigma, mob, steps, checkpoint_every=20)
        loss = 0.5 * g.h ** 2 * ((out[0] - target) ** 2).sum()
        _sync()
        t1 = time.perf_counter()
        loss.backward()
        _sync()
        t2 = time.perf_counter()
        fwd_s.append(t1 - t0)
        bwd_s.append(t2 - t1)
    tf, tb = min(fwd_s), min(bwd_s)
    return {"workload": "oscillating_drop_128^2_fp64", "steps": steps, "checkpoint_every": 20,
            "forward_ms": round(tf * 1e3, 2), "backward_ms": round(tb * 1e3, 2),
            "adjoint_over_forward": round(tb / tf, 3), "repeats": 3,
            "dL_dsigma": float(sigma.grad), "dL_dM": float(mob.grad)}


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

    if args.calibrate_copy:
        # reference kernel for the HBM byte counters: reads and writes 256 MiB
        a = torch.empty(32 << 20, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

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
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": recorded_traffic(dom["name"]),
                "kernel": dom["name"], "avg_us": round(dom["ms"] * 1e3 / dom["launches"], 3),
                "bytes_per_launch": round(dom["bytes"] / dom["launches"], 1),
                "launches_per_step": round(dom["launches"] / args.profile_steps, 1),
                "share_of_kernel_time": round(dom["ms"] / sum(k["ms"] for k in kernels), 4)}
        if dom["name"] == "coarse_solve":
            roof["note"] = ("one-workgroup V-cycle of the levels of <= 2048 cells out of LDS: ~45 dependent "
                            "LDS passes on one CU, latency-bound; its HBM bytes are the copy-in and the "
                            "write-back of x")

    cpu = None
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        cpu = cpu_baseline(prob, args.cpu_steps)

    secondary = None
    extras = [e for e in args.extras.split(",") if e] if not args.no_extras else []
    unknown = set(extras) - {"precision_form", "batched", "adjoint"}
    if unknown:
        print("unknown --extras entries: %s" % ", ".join(sorted(unknown)), file=sys.stderr)
        sys.exit(2)
    if extras:
        del g, st
        secondary = {}
        runs = {"precision_form": lambda: bench_precision_form(P, W, args.extra_steps),
                "batched": lambda: bench_batched(P, W, args.extra_steps),
                "adjoint": lambda: bench_adjoint(P, W)}
        for name in ("precision_form", "batched", "adjoint"):
            if name in extras:
                torch.cuda.empty_cache()
                secondary[name] = runs[name]()

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
        "secondary": secondary,
    }
    if kernels is not None:
        out["kernels"] = [{"name": k["name"], "launches": k["launches"], "ms": round(k["ms"], 3),
                           "GBs": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 1)} for k in
                          sorted(kernels, key=lambda r: -r["ms"])]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
