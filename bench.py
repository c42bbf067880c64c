"""Benchmark of the shallow-water step on one MI355X.

Default workload: the valley flood (4M-triangle Delaunay mesh of a jittered
lattice over a 20 km x 4 km synthetic DEM with a meandering channel), fully
wet snapshot (1 m of water moving at 0.5 m/s), FP32 state with FP64
thresholds / dt / mass, stepped through hipGraph launches of the C-ABI
library.  A step is one full pass of the method over every cell
(reconstruction, HLLC, update, friction, positivity, next-dt reduction).

Prints one JSON line: cell-updates/s, the roofline object of the step kernel
(algorithmic bytes per cell-update x cells / kernel time, timed with HIP events
on the library's stream) and the FP64 oracle timed on a bounded sample on the
host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell-update: every array element of the step moved
# once (state in, geometry, neighbour ids, state out), gathers from cache
ALGO_BYTES = {"fp32": 72.0, "fp64": 132.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import swe_inputs as S
    from gpu_util import cached
    if name == "valley_wet":
        return cached("valley", S.valley_flood, n_cells=4_000_000, snapshot="wet")
    if name == "valley_dry":
        return cached("valley", S.valley_flood, n_cells=4_000_000)
    if name == "lake":
        return cached("lake", S.lake_at_rest, n_cells=200_000)
    raise SystemExit(f"unknown workload {name}")


def time_gpu(sc, precision, steps, warmup, autotune=True):
    import torch
    from paper_2102_12862_amd import swe
    dev = swe.TorchDevice()
    mesh = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=dev)
    p = swe.FP32 if precision == "fp32" else swe.FP64
    st = swe.State(mesh, sc, precision=p)
    tune = None
    if autotune:
        tune = st.autotune(k=5)
    st.launch_steps(warmup)
    st.sync()
    stream = dev.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    st.launch_steps(steps)
    e1.record(stream)
    st.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    m = st.mass()
    st.close()
    mesh.close()
    return dict(ms=ms, wall=wall, tune=tune, mass=m)


def time_oracle(sc, budget_s=15.0, max_steps=50):
    import oracle
    t0 = time.perf_counter()
    mesh = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    sim = oracle.Sim(sc, mesh=mesh)
    prep = time.perf_counter() - t0
    n = 0
    t0 = time.perf_counter()
    while n < max_steps and time.perf_counter() - t0 < budget_s:
        sim.step()
        n += 1
    el = time.perf_counter() - t0
    return dict(steps=n, seconds=el, prep=prep, rate=sc.n_cells * n / el)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="valley_wet")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path is one device's share of the mesh; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    log(f"[bench] generating {args.workload}")
    t0 = time.perf_counter()
    sc = make_workload(args.workload)
    log(f"[bench] {sc.name}: {sc.n_cells} cells ({time.perf_counter() - t0:.1f}s)")
    r = time_gpu(sc, args.precision, args.steps, args.warmup, autotune=not args.no_autotune)
    ms_step = r["ms"] / args.steps
    N = sc.n_cells
    value = N * args.steps / (r["ms"] * 1e-3)
    achieved = ALGO_BYTES[args.precision] * N / (ms_step * 1e-3) / 1e9
    log(f"[bench] gpu {args.precision}: {ms_step * 1e3:.1f} us/step, {value:.3e} cell-updates/s, tune {r['tune']}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle sample")
        o = time_oracle(sc)
        cpu = {"value": o["rate"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{o['steps']} FP64 steps of the same {N}-cell workload ({o['seconds']:.1f}s, serial C)"}
        log(f"[bench] oracle {o['rate']:.3e} cell-updates/s")
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": sc.name, "cells": N, "precision": args.precision,
                   "block_size_cells_per_thread": r["tune"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_cell": ALGO_BYTES[args.precision]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
