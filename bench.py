#!/usr/bin/env python3
"""Benchmark of the split CHNS time step on one MI355X.

Headline workload: the three-phase drops, 128^3 periodic cells (8 drops of
each of two phases in a carrier phase, seeded radii 0.05-0.12, pairwise
surface tensions U[0.5, 1.5], densities 100 / 10 / 1, divergence-free
velocity perturbation of amplitude 1e-2), in two arithmetic forms on the same
input:
  fp64         FP64 throughout, at the solver tolerances the oracle parity
               tests use (CH 1e-15, momentum 1e-13, pressure 1e-12)
  fp32_refine  the precision form: FP32 multigrid preconditioner inside FP64
               CG (FP64 vectors, operator apply and dots), at its own tolerances
               (1e-10 / 1e-9 / 1e-8; its state stays within 1.5e-8 of the FP64
               run over the configuration's 500 steps, budget 1e-5)
A step is one full pass T1..T9 (two CH solves, three momentum components,
pressure projection).  By default each form runs the configuration's 500
steps from the initial state, 10 untimed and 490 timed.  Inputs are
synthetic and already resident in device memory when the timed region
starts.  `value` is the precision form's throughput; the FP64 form's and the
ratio are in `config`.

Secondary measurements (key "secondary", each on its own workload, skipped
with --no-extras):
  bubble        2D rising bubble 256 x 512, FP64, its dominant kernel class
  hbm_sweeps    one pressure solve on a 512^3 (FP64) and an 8192^2 (FP64)
                grid: per kernel class achieved GB/s where every level-0
                sweep touches far more than the 256 MB Infinity Cache
  batched       ensemble of 512 oscillating drops (64^2 .. 256^2), FP32 +
                refinement, autotuned form; eager and hipGraph-captured steps
  adjoint       oscillating drop 128^2, FP64: checkpointed backward vs
                forward time

Prints one JSON line:
  value         grid cell-updates/s = cells * steps / wall-time of the timed
                region (host clock after a device synchronisation on both
                sides; hipEvents on the library stream agree)
  roofline      the kernel class with the largest share of device time in a
                separate instrumented pass of the headline form (hipEvent pair
                recorded by the dispatch of every launch on the library
                stream): algorithmic bytes / kernel time vs the 8 TB/s HBM peak;
                traffic = the committed FETCH_SIZE + WRITE_SIZE counter record
  cpu_baseline  the CPU oracle (numpy / scipy, FP64, one thread) on a bounded
                sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid cell-updates/s per time step (FP64 vs FP32+refine), %HBM roofline, adjoint/fwd"
HBM_PEAK_GBS = 8000.0
EXTRAS = ("bubble", "hbm_sweeps", "batched", "adjoint")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # default: the headline configuration's 500 steps, 10 untimed and 490 timed
    ap.add_argument("--steps", type=int, default=490)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-headline", action="store_true", help="skip the headline legs (profiling runs of extras)")
    ap.add_argument("--headline-forms", default="fp64,fp32_refine",
                    help="headline forms to run (profiling runs take one form each)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated secondary measurements to run (subset of the default)")
    ap.add_argument("--serial-components", action="store_true",
                    help="run the momentum components one after another on the grid's stream (kernel profiles)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for the HBM byte counters)")
    ap.add_argument("--hbm-shapes", default="512^3,8192^2", help="grids of the hbm_sweeps measurement")
    ap.add_argument("--batched-form", default="auto",
                    help="batched leg: 'auto' (autotuned), 'tiled:TILE_CELLS' or 'persistent:THREADS:BLOCKS' "
                         "(fixed form, no autotuning: profiling runs)")
    ap.add_argument("--traffic-from", nargs="+", metavar="WORKLOAD=FETCH_CSV,WRITE_CSV",
                    help="no GPU run: build profiles/traffic.json from rocprofv3 --pmc counter CSVs of bench.py "
                         "runs (one FETCH_SIZE and one WRITE_SIZE pass per workload, each with --calibrate-copy)")
    ap.add_argument("--dispatch-table", nargs=3, metavar=("TRACE_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: per kernel and launch size, mean duration and counter bytes per dispatch "
                         "(the largest --top entries by total time)")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--durations-from", nargs="+", metavar="WORKLOAD=KERNEL_TRACE_CSV",
                    help="no GPU run: print per kernel class dispatch counts and mean durations from rocprofv3 "
                         "--kernel-trace CSVs, with the class filters of --traffic-from")
    return ap.parse_args()


def recorded_traffic(workload, kernel_class):
    """HBM bytes per launch of a kernel class on a workload (dispatch-weighted
    over its kernels) from the committed counter record (two rocprofv3 --pmc
    passes, FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size);
    None if the record holds no such class or the sources of the library
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])).hexdigest()
        if h != rec["sources_sha256"]:
            return None
        for r in rec["records"]:
            if r["workload"] == workload and r["kernel_class"] == kernel_class:
                return r["traffic_bytes_per_launch"]
        return None
    except (OSError, ValueError, KeyError):
        return None


# Kernel classes of the library's per-kernel timing, by kernel name (the
# template arguments after the name are matched by the workload filters).
KERNEL_CLASSES = {
    "smooth": ("k_presmooth_pair", "k_presmooth", "k_gs_color", "k_presmooth_march", "k_gs_color_march", "k_gs_red_rz"),
    "residual": ("k_residual", "k_residual_march"),
    "restrict": ("k_restrict3_lds", "k_restrict3_pair", "k_restrict"),
    "prolong": ("k_prolong_add3",),
    "coarse_solve": ("k_vcycle_lds", "k_vcycle_block"),
    "mg_down": ("k_down_tile2", "k_down_tile2_cg", "k_down3_tile"),
    "mg_up": ("k_up_tile2", "k_up_tile2_cg", "k_up3_tile"),
    "pcg_apply": ("k_pcg_apply3_march", "k_pcg_apply_slot", "k_pcg_ch_lap", "k_pcg_ch_apply"),
    "pcg_update": ("k_pcg_update", "k_pcg_fin_rr"),
    "pcg_dot": ("k_pcg_rz",),
    # the batched tiled form (one launch per sweep over the tiles of all problems)
    "t_down": ("k_t_down2",),
    "t_up": ("k_t_up2",),
    "t_apply": ("k_t_apply",),
    "t_update": ("k_t_update", "k_t_fin_rr"),
    "t_dot": ("k_t_rz", "k_t_fin_rz"),
    "t_small_levels": ("k_t_vcycle_small_lds", "k_t_vcycle_small"),
    "t_sweep": ("k_t_sweep", "k_t_restrict"),
    "t_phase": ("k_t_phase",),
    "ch_spectral": ("k_axis_mfma64", "k_axis_gemm", "k_axis_gemm16s", "k_spectral_scale_batch", "k_spectral_scale",
                    "k_axis_fft"),
    # the step's own passes and the solver set-ups
    "ch_rhs": ("k_ch_rhs", "k_ch_rhs3", "k_cn_ch_rhs"),
    "mu": ("k_mu", "k_mu3"),
    "phi_update": ("k_phi_update", "k_phi_update3", "k_cn_phi_update"),
    "mom_setup": ("k_mom_setup", "k_mom_setup_all", "k_mom_setup3_all", "k_mom_setup_walls", "k_mflux3",
                  "k_velocity_guess", "k_cn_mom_setup"),
    "p_setup": ("k_p_setup", "k_p_setup3", "k_p_coef_rho", "k_pressure_guess"),
    "project": ("k_project", "k_project3", "k_cn_project", "k_cn_finish"),
    "mg_setup": ("k_coarsen", "k_conv_coef", "k_fill_ch", "k_invd", "k_setup_block"),
    "pcg_init": ("k_pcg_init_slot", "k_pcg_init_zero", "k_pcg_init_ch", "k_pcg_fin_init", "k_round_vec",
                 "k_ch_lap_plain", "k_cn_zero"),
    "mean": ("k_sum", "k_sub_mean"),
}

# Which dispatches of a profiled bench.py run belong to a workload: every
# workload, each headline form included (--headline-forms), is profiled in a
# bench.py run of its own.
WORKLOAD_FILTERS = {
    "ternary_drops3d_128^3_fp32_refine": lambda args: True,
    "ternary_drops3d_128^3_fp64": lambda args: True,
    "rising_bubble_256x512_fp64": lambda args: True,
    "pressure_512^3_fp64": lambda args: True,
    "pressure_8192^2_fp64": lambda args: True,
    "ensemble_512_fp32_refine": lambda args: True,
}
# the counter record stands for the library built from these sources
TRAFFIC_SOURCES = sorted("paper_2009_06628_amd/csrc/" + f for f in os.listdir(os.path.join(ROOT, "paper_2009_06628_amd",
                                                                                          "csrc"))
                         if f.endswith((".hip", ".h")))


def _class_of(kernel_name):
    """(class, template arguments) of a rocprofv3 kernel name, or None.  The
    template arguments are the text of the first <...> after the name (empty
    for a kernel that is not a template)."""
    name = kernel_name.strip()
    head = name.split("(")[0]
    base, _, rest = head.partition("<")
    base = base.strip().split()[-1].split("::")[-1] if base.strip() else ""
    depth, targs = 1, ""
    for ch in rest:
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
            if depth == 0:
                break
        targs += ch
    for cls, names in KERNEL_CLASSES.items():
        if base in names:
            return cls, targs
    return None


def _read_csv(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _counter_rows(path, counter):
    """(kernel name, value in bytes) per dispatch of a --pmc CSV in dispatch
    order (the counter is reported in KiB)."""
    rows = []
    for r in _read_csv(path):
        if r.get("Counter_Name", counter) != counter:
            continue
        rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
    rows.sort()
    return [(k, v) for (_, k, v) in rows]


def build_traffic(specs):
    """profiles/traffic.json from FETCH_SIZE / WRITE_SIZE CSVs.  Each pass ran
    bench.py with --calibrate-copy: the copy of 256 MiB (read and write) that
    starts the run fixes the scale of each counter."""
    import hashlib
    records = []
    scales = {}
    for spec in specs:
        workload, files = spec.split("=", 1)
        fetch_csv, write_csv = files.split(",")
        filt = WORKLOAD_FILTERS[workload]
        per = {}
        for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
            rows = _counter_rows(path, counter)
            # the calibration copy is the run's first buffer copy (--calibrate-copy
            # issues it before anything else touches the device)
            copy = [v for (k, v) in rows if "copyBuffer" in k]
            ref = 256.0 * 1024 * 1024
            scale = ref / copy[0] if copy and copy[0] > 0 else 1.0
            scales.setdefault(workload, {})[counter] = round(scale, 5)
            for k, v in rows:
                c = _class_of(k)
                if c is None or not filt(c[1]):
                    continue
                d = per.setdefault(c[0], {"kernels": set(), "FETCH_SIZE": [], "WRITE_SIZE": []})
                d["kernels"].add(k.split("(")[0].strip())
                d[counter].append(v * scale)
        for cls, d in sorted(per.items()):
            n = min(len(d["FETCH_SIZE"]), len(d["WRITE_SIZE"]))
            if n == 0:
                continue
            fetch = sum(d["FETCH_SIZE"]) / len(d["FETCH_SIZE"])
            write = sum(d["WRITE_SIZE"]) / len(d["WRITE_SIZE"])
            records.append({"workload": workload, "kernel_class": cls, "kernels": sorted(d["kernels"]),
                            "dispatches": n, "fetch_bytes_per_dispatch": round(fetch, 1),
                            "write_bytes_per_dispatch": round(write, 1),
                            "traffic_bytes_per_launch": round(fetch + write, 1)})
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in TRAFFIC_SOURCES)).hexdigest()
    rec = {"counter_scales": scales, "records": records, "sources": TRAFFIC_SOURCES, "sources_sha256": h}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"written": "profiles/traffic.json", "records": len(records), "scales": scales}))


def print_durations(specs):
    """Per kernel class: dispatches and mean duration (us) from --kernel-trace
    CSVs, with the workload filters."""
    for spec in specs:
        workload, path = spec.split("=", 1)
        filt = WORKLOAD_FILTERS[workload]
        per = {}
        for r in _read_csv(path):
            c = _class_of(r["Kernel_Name"])
            if c is None or not filt(c[1]):
                continue
            dur = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3
            d = per.setdefault(c[0], [0, 0.0])
            d[0] += 1
            d[1] += dur
        print(json.dumps({"workload": workload,
                          "classes": {k: {"dispatches": v[0], "mean_us": round(v[1] / v[0], 3),
                                          "total_ms": round(v[1] / 1e3, 3)} for k, v in sorted(per.items())}}))


def print_dispatch_table(trace_csv, fetch_csv, write_csv, top):
    """Per kernel and launch size (grid threads): dispatches and mean duration
    from a --kernel-trace CSV and mean FETCH_SIZE + WRITE_SIZE bytes per
    dispatch from two --pmc CSVs of the same command run with --calibrate-copy
    (scaled by the run's first buffer copy).  The three runs issue the same
    dispatch sequence, so the k-th dispatch of a kernel in the trace is paired
    with its k-th dispatch in each counter pass.  Grid-stride kernels cap their
    grid, so several levels can share a launch size: each group is also
    reported for its largest launches alone (duration >= half the group's
    longest).  The `top` groups with the largest total time."""
    def by_name(rows, value):
        out = {}
        for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
            out.setdefault(r["Kernel_Name"].split("(")[0].replace("void ", "").strip(), []).append(value(r))
        return out

    trace = by_name(_read_csv(trace_csv), lambda r: (
        int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]),
        (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3))
    counters = []
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _read_csv(path) if r.get("Counter_Name", counter) == counter]
        first_copy = min((r for r in rows if "copyBuffer" in r["Kernel_Name"]), key=lambda r: int(r["Dispatch_Id"]),
                         default=None)
        scale = 1.0
        if first_copy is not None and float(first_copy["Counter_Value"]) > 0:
            scale = 256.0 * 1024 * 1024 / (float(first_copy["Counter_Value"]) * 1024.0)
        counters.append(by_name(rows, lambda r, sc=scale: float(r["Counter_Value"]) * 1024.0 * sc))
    groups = {}
    for name, seq in trace.items():
        f, w = counters[0].get(name, []), counters[1].get(name, [])
        paired = len(f) == len(seq) and len(w) == len(seq)
        for k, (grid, dur) in enumerate(seq):
            groups.setdefault((name, grid), []).append((dur, f[k] + w[k] if paired else None))
    out = []
    for (name, grid), rows in sorted(groups.items(), key=lambda kv: -sum(d for d, _ in kv[1]))[:top]:
        def summary(sel):
            n = len(sel)
            mean = sum(d for d, _ in sel) / n
            byts = [b for _, b in sel if b is not None]
            traffic = sum(byts) / len(byts) if len(byts) == n else None
            return {"dispatches": n, "mean_us": round(mean, 3), "counter_bytes": round(traffic) if traffic else None,
                    "counter_TBs": round(traffic / mean / 1e6, 3) if traffic else None}
        longest = max(d for d, _ in rows)
        out.append({"kernel": name, "grid_threads": grid, "all": summary(rows),
                    "largest": summary([r for r in rows if r[0] >= 0.5 * longest])})
    print(json.dumps(out, indent=0))


def _sync():
    import torch
    torch.cuda.synchronize()


def roofline_of(kernels, steps, workload):
    """Roofline object of the kernel class with the most device time."""
    dom = max(kernels, key=lambda r: r["ms"])
    achieved = dom["bytes"] / (dom["ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": recorded_traffic(workload, dom["name"]),
            "kernel": dom["name"], "avg_us": round(dom["ms"] * 1e3 / dom["launches"], 3),
            "bytes_per_launch": round(dom["bytes"] / dom["launches"], 1),
            "launches_per_step": round(dom["launches"] / steps, 1),
            "share_of_kernel_time": round(dom["ms"] / sum(k["ms"] for k in kernels), 4)}


def kernel_table(kernels):
    return [{"name": k["name"], "launches": k["launches"], "ms": round(k["ms"], 3),
             "GBs": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 1)} for k in sorted(kernels, key=lambda r: -r["ms"])]


def timed_run(P, prob, precision, warmup, steps, serial):
    """Warm-up, then `steps` timed steps; returns the grid, the state and the
    timings (wall clock and hipEvents on the library stream)."""
    import torch
    import workloads as W
    g = P.grid_for_problem(prob, precision, device="cuda:0")
    if serial:
        g.set_option(P.CHNS_OPT_SERIAL_COMPONENTS, 1)
    st = g.new_state(W.initial_state(prob))
    if warmup:
        g.step(st, warmup, stats=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(g.stream)
    g.step(st, steps, stats=False)
    e1.record(g.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return g, st, {"wall": wall, "event_s": e0.elapsed_time(e1) / 1e3}


def instrumented(g, st, steps, workload):
    g.set_timing(True)
    g.step(st, steps, stats=False)
    _sync()
    kernels = g.get_timing()
    g.set_timing(False)
    return kernels, roofline_of(kernels, steps, workload)


def bench_bubble(P, W, steps, warmup, profile_steps, serial):
    """2D rising bubble, FP64 (latency-bound: ~30 MB working set)."""
    prob = W.rising_bubble(256, steps=2000)
    g, st, t = timed_run(P, prob, P.CHNS_FP64, warmup, steps, serial)
    stats = g.step(st, 1)
    out = {"workload": "rising_bubble_256x512_fp64", "cells": prob.cells, "steps": steps,
           "value": round(prob.cells * steps / t["wall"], 1), "ms_per_step": round(t["wall"] / steps * 1e3, 4),
           "event_seconds": round(t["event_s"], 4),
           "iters_last_step": {"ch": stats["iters_ch"], "mom": stats["iters_mom"], "p": stats["iters_p"]}}
    if profile_steps:
        kernels, roof = instrumented(g, st, profile_steps, out["workload"])
        out["roofline"] = roof
        out["kernels"] = kernel_table(kernels)[:8]
    return out


def bench_hbm_sweeps(P, W, hbm_shapes):
    """One pressure solve (rtol 1e-10) on grids whose level-0 arrays are far
    larger than the Infinity Cache: 512^3 FP64 (1.07 GB per array) and
    8192^2 FP64 (0.54 GB per array); density ratio 10 drop.  Per kernel class:
    launches, ms, achieved GB/s (algorithmic bytes / kernel time)."""
    import numpy as np
    import torch
    out = {}
    shapes = {"512^3": (512, 512, 512), "8192^2": (8192, 8192)}
    for key in [x for x in hbm_shapes.split(",") if x]:
        n = shapes[key]
        name = "pressure_%s_fp64" % key
        h = 1.0 / n[0]
        g = P.create_grid(n, h, ("periodic",) * len(n), device="cuda:0")
        dev = torch.device("cuda:0")
        axes = [(torch.arange(m, dtype=torch.float64, device=dev) + 0.5) * h for m in reversed(n)]
        X = torch.meshgrid(*axes, indexing="ij")
        r = torch.sqrt(sum((x - 0.5) ** 2 for x in X))
        del X
        phi = torch.tanh((r - 0.25) / (2 ** 0.5 * 1.5 * h))
        del r
        rho = 0.55 + 0.45 * phi
        gen = torch.Generator(device=dev).manual_seed(7)
        rhs = torch.randn(rho.shape, dtype=torch.float64, device=dev, generator=gen)
        del phi
        p = torch.zeros_like(rho)
        g.solve_pressure(rho, rhs, p, rtol=1e-10, max_iter=200)    # warm-up (first-use costs)
        _progress("hbm_sweeps %s: warm-up solve done" % key)
        p.zero_()
        _sync()
        g.set_timing(True)
        res = g.solve_pressure(rho, rhs, p, rtol=1e-10, max_iter=200)
        _sync()
        kernels = g.get_timing()
        g.set_timing(False)
        cells = int(np.prod(n))
        out[name] = {"cells": cells, "iters": res["iters"], "rel_res": res["rel_res"],
                     "bytes_per_array": 8 * cells,
                     "kernels": [dict(k, traffic=recorded_traffic(name, k["name"])) for k in kernel_table(kernels)]}
        del g, rho, rhs, p
        torch.cuda.empty_cache()
    return out


def _progress(msg):
    """One line on stderr when a phase of the run ends (profiled runs are slow
    and print their JSON line only at the end)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def bench_batched(P, W, steps, form="auto", cpu_problems=0):
    """Batched ensemble: 512 problems, precision form; autotuned form and
    launch shape (or a fixed one); timed eagerly (solves run to convergence
    with host checks) and as a captured hipGraph (fixed per-solve iteration
    budgets).  cpu_problems > 0: the oracle's step on the first members of the
    ensemble as its CPU baseline."""
    probs = W.ensemble(count=512, seed=4, steps=200, **W.PRECISION_FORM_TOLERANCES)
    b = P.create_batch(probs, P.CHNS_FP32_REFINE, device="cuda:0")
    st = b.new_state([W.initial_state(p) for p in probs])
    _progress("batched: %d problems created" % len(probs))
    out = {"workload": "ensemble_512_oscillating_drops_fp32_refine", "problems": len(probs),
           "cells": b.total_cells, "steps": steps}
    if form == "auto":
        tune = b.autotune(st, 1)
        out.update({"form": tune["mode"], "tile_cells": tune["tile_cells"], "graph_budgets": list(tune["budgets"]),
                    "autotune_ms_per_step": {"%s_%d_%d" % (c[0], c[1], c[2]): round(c[3], 2)
                                             for c in tune["candidates"]}})
    else:
        parts = form.split(":")
        if parts[0] == "tiled":
            b.set_tiled(int(parts[1]))
        else:
            b.set_launch(int(parts[1]), int(parts[2]))
        out.update({"form": parts[0], "launch": [int(x) for x in parts[1:]]})
    for label, graph in (("eager", False), ("graph", True)):
        b.step(st, steps, use_graph=graph, stats=False)     # warm-up (and capture)
        _sync()
        _progress("batched: %s warm-up done" % label)
        t0 = time.perf_counter()
        stats = b.step(st, steps, use_graph=graph, stats=True)
        dt = time.perf_counter() - t0
        _progress("batched: %s steps done" % label)
        tot = sum(s["total_iters"] for s in stats)
        out[label] = {"value": round(b.total_cells * steps / dt, 1), "ms_per_step": round(dt / steps * 1e3, 3),
                      "pcg_iterations_per_problem_step": round(tot / (len(probs) * steps), 2),
                      "unconverged": sum(1 for s in stats if s["flags"])}
    out["value"] = out["graph"]["value"]
    out["ms_per_step"] = out["graph"]["ms_per_step"]
    if cpu_problems > 0:
        out["cpu_baseline"] = cpu_baseline_batched(probs[:cpu_problems])
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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(prob, steps):
    """The three-phase oracle on the host: `steps` steps of the same 128^3
    workload from its initial state, one thread (no warm-up step: one step
    takes about a minute)."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import MACGrid
    from oracle import ternary as T

    g = MACGrid(prob.n, prob.h, prob.periodic)
    prm = T.Params3.from_props(prob.props)
    st = W.initial_state(prob)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(steps):
            st = T.step3(g, st, prm)
        dt = time.perf_counter() - t0
    return {"value": round(prob.cells * steps / dt, 1), "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d step(s) of the %dx%dx%d three-phase drops from the initial state, FP64, one thread "
                      "(%.1f s; host CPU: %s, %d logical CPUs)"
                      % (steps, prob.n[0], prob.n[1], prob.n[2], dt, _cpu_model(), os.cpu_count() or 0)}


def cpu_baseline_batched(probs):
    """The two-phase oracle on the host: one step of each given member of the
    ensemble from its initial state, one thread."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import MACGrid, Params
    from oracle import chns as C

    cells = sum(p.cells for p in probs)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for p in probs:
            C.step(MACGrid(p.n, p.h, p.periodic), W.initial_state(p), Params.from_props(p.props))
        dt = time.perf_counter() - t0
    sizes = sorted(set(p.n[0] for p in probs))
    return {"value": round(cells / dt, 1), "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "one step of each of the first %d members of the 512-problem ensemble (n in %s, %d cells), "
                      "FP64, one thread (%.1f s; host CPU: %s, %d logical CPUs)"
                      % (len(probs), sizes, cells, dt, _cpu_model(), os.cpu_count() or 0)}


def main():
    args = parse()
    if args.dispatch_table:
        print_dispatch_table(*args.dispatch_table, args.top)
        return
    if args.traffic_from or args.durations_from:
        if args.traffic_from:
            build_traffic(args.traffic_from)
        if args.durations_from:
            print_durations(args.durations_from)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2009_06628_amd as P
    import workloads as W

    extras = [e for e in args.extras.split(",") if e] if not args.no_extras else []
    unknown = set(extras) - set(EXTRAS)
    if unknown:
        print("unknown --extras entries: %s" % ", ".join(sorted(unknown)), file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        # reference kernel for the HBM byte counters: reads and writes 256 MiB
        a = torch.empty(32 << 20, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    workload = "ternary_drops3d_128^3"
    out = {"metric": METRIC, "value": None, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic", "config": None, "roofline": None,
           "cpu_baseline": None}
    prob = None
    if not args.no_headline:
        prob = W.ternary_drops3d(128, steps=500)
        legs = {}
        states = {}
        forms = [f for f in args.headline_forms.split(",") if f]
        for name, prec, pr in (("fp64", P.CHNS_FP64, prob),
                               ("fp32_refine", P.CHNS_FP32_REFINE,
                                W.ternary_drops3d(128, steps=500, **W.PRECISION_FORM_TOLERANCES))):
            if name not in forms:
                continue
            g, st, t = timed_run(P, pr, prec, args.warmup, args.steps, args.serial_components)
            _progress("headline %s: timed steps done" % name)
            stats = g.step(st, 1)     # outside the timed region: solver statistics and diagnostics
            legs[name] = {"value": round(prob.cells * args.steps / t["wall"], 1),
                          "ms_per_step": round(t["wall"] / args.steps * 1e3, 4),
                          "event_seconds": round(t["event_s"], 4),
                          "tolerances": {"ch": pr.props.rtol_ch, "mom": pr.props.rtol_mom, "p": pr.props.rtol_p},
                          "iters_last_step": {"ch": stats["iters_ch"], "mom": stats["iters_mom"],
                                              "p": stats["iters_p"]},
                          "mass_phase": stats["mass_phase"], "energy": stats["energy"]}
            if not args.no_profile and args.profile_steps > 0:
                kernels, roof = instrumented(g, st, args.profile_steps, workload + "_" + name)
                legs[name]["roofline"] = roof
                legs[name]["kernels"] = kernel_table(kernels)
            states[name] = st
            del g
            torch.cuda.empty_cache()
        diff = None
        if len(states) == 2:
            a, b = states["fp32_refine"], states["fp64"]
            diff = 0.0
            for i in range(2):
                diff = max(diff, float((a["phi"][i] - b["phi"][i]).abs().max() / b["phi"][i].abs().max()))
            for d in range(3):
                diff = max(diff,
                           float((a["u"][d] - b["u"][d]).abs().max() / b["u"][d].abs().max().clamp_min(1e-300)))
            del a, b
        del states
        torch.cuda.empty_cache()
        f64, f32 = legs.get("fp64"), legs.get("fp32_refine")
        head = f32 if f32 is not None else f64
        out.update(value=head["value"], ms_per_step=head["ms_per_step"], roofline=head.pop("roofline", None))
        out["config"] = {"workload": workload, "grid": list(prob.n), "cells": prob.cells, "bc": list(prob.bc),
                         "nphases": 3, "densities": list(prob.props.rho3), "viscosities": list(prob.props.eta3),
                         "surface_tensions": [round(x, 6) for x in prob.props.sigma3], "Re": prob.props.Re,
                         "dt": prob.props.dt, "form": "fp32_refine" if f32 is not None else "fp64",
                         "fp32_refine": f32, "fp64": f64,
                         "speedup_fp32_refine_vs_fp64": round(f32["value"] / f64["value"], 3) if f32 and f64 else None,
                         "max_rel_state_diff_fp32_refine_vs_fp64": diff,
                         "serial_components": bool(args.serial_components)}
        if not args.no_cpu_baseline and args.cpu_steps > 0:
            out["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)

    if extras:
        secondary = {}
        runs = {"bubble": lambda: bench_bubble(P, W, 2000 if args.steps >= 100 else args.steps, args.warmup,
                                               args.profile_steps if not args.no_profile else 0,
                                               args.serial_components),
                "hbm_sweeps": lambda: bench_hbm_sweeps(P, W, args.hbm_shapes),
                "batched": lambda: bench_batched(P, W, args.extra_steps, args.batched_form,
                                                 0 if args.no_cpu_baseline else 16),
                "adjoint": lambda: bench_adjoint(P, W)}
        for name in EXTRAS:
            if name in extras:
                torch.cuda.empty_cache()
                secondary[name] = runs[name]()
                _progress("%s done" % name)
        out["secondary"] = secondary
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
