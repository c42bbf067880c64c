"""Benchmark of the shallow-water step on one MI355X.

Headline workload: the valley flood (4M-triangle Delaunay mesh of a jittered
lattice over a 20 km x 4 km synthetic DEM with a meandering channel), fully
wet snapshot (1 m of water moving at 0.5 m/s, so every cell does the whole
step), FP32 state with FP64 depth tests / dt / mass, stepped through hipGraph
launches of the C-ABI library.  A step is one full pass of the method over
every cell: reconstruction, HLLC, update, friction, positivity and the
device-side CFL reduction.

Prints one JSON line: cell-updates/s, the roofline object of the step kernel
(algorithmic bytes per cell-update x cells / kernel time, timed with HIP events
on the library's stream), the FP64 oracle timed on a bounded sample on the
host, and (under "variants") the same metric in FP64, on the 200k-cell lake,
for a batched ensemble against the same members solved one after another, and
for a served Poisson request trace (p50/p99 latency) against one-at-a-time
serving.
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
# once (state in, bed, g n^2, cell area, 3 neighbour ids, 3 l*n pairs, state
# out), neighbour gathers served from cache
ALGO_BYTES = {"fp32": 72.0, "fp64": 132.0}
# each passive species adds its specific mass in and out
SPECIES_BYTES = {"fp32": 8.0, "fp64": 16.0}


# HBM traffic of the step kernel, measured with the FETCH_SIZE and WRITE_SIZE
# counters (each scaled by what it reads for a plain copy of known size); it
# is reported only while the kernel sources still hash to the digest recorded
# with the measurement
def traffic_profile(precision, species, morpho=False):
    kern = "k_step_morpho" if morpho else f"k_step_species{species}" if species else "k_step"
    return os.path.join(ROOT, "profiles", f"{kern}_{precision}_valley4m_hbm_traffic.md")


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2102_12862_amd", "csrc", f)
                  for f in ("kernels.hip", "swe_internal.h", "meshprep.cpp", "meshprep.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, tile, species=0, morpho=False):
    """Bytes per step-kernel launch from the committed counter profile, or
    None when it was taken on other kernel sources or another configuration."""
    try:
        with open(traffic_profile(precision, species, morpho)) as fh:
            kv = dict(line.strip()[2:].split(": ", 1) for line in fh if line.startswith("- ") and ": " in line)
    except OSError:
        return None
    try:
        if (kv.get("kernel_digest") != kernel_digest() or kv.get("workload") != workload
                or kv.get("precision") != precision):
            return None
        return float(kv[f"traffic_bytes_per_launch_tile{tile}"])
    except (KeyError, ValueError):
        return None


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


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def species_phi0(sc, ns):
    """Initial concentrations of ns species: a front across the domain at
    the median centroid x, then uniform backgrounds."""
    cx = sc.centroids()[:, 0]
    rows = [np.where(cx < np.median(cx), 1.0, 0.0)] + [np.full(sc.n_cells, 0.1 * (k + 1)) for k in range(ns - 1)]
    return np.stack(rows[:ns])


def time_gpu(sc, precision, steps, warmup, autotune=True, species=0, tile=0, morpho=False):
    """Kernel time per step over `steps` graph-launched steps."""
    import torch
    from paper_2102_12862_amd import swe
    from gpu_util import device
    dev = device()
    mesh = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=dev)
    p = swe.FP32 if precision == "fp32" else swe.FP64
    st = swe.State(mesh, sc, precision=p, steps_per_graph=50, block_size=tile)
    if species:
        st.set_scalars(species_phi0(sc, species))
    if morpho:
        import swe_inputs as S
        st.set_morpho(S.Morpho("mpm"))
    tune = st.autotune(k=5) if (autotune and not tile) else None
    st.launch_steps(warmup)
    st.sync()
    e0, e1 = _events()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(dev.stream)
    st.launch_steps(steps)
    e1.record(dev.stream)
    st.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    st.close()
    mesh.close()
    return dict(ms=ms, wall=wall, tune=tune, ms_step=ms / steps, rate=sc.n_cells * steps / (ms * 1e-3))


def time_oracle(sc, budget_s=15.0, max_steps=50, precision="fp32"):
    """The FP64 oracle on a bounded sample of the workload (steps with the
    time step fixed at half the initial CFL step), then the GPU path on the
    same steps: the oracle's rate, and the GPU's max and L1 errors in h, qx,
    qy against it."""
    import oracle
    from gpu_util import device, errors
    from paper_2102_12862_amd import swe
    import swe_inputs as S
    t0 = time.perf_counter()
    mesh = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    fixed = S.Scenario(**{**sc.__dict__})
    fixed.dt_max = 0.5 * oracle.Sim(sc, mesh=mesh).next_dt()
    sim = oracle.Sim(fixed, mesh=mesh)
    prep = time.perf_counter() - t0
    n = 0
    t0 = time.perf_counter()
    while n < max_steps and time.perf_counter() - t0 < budget_s:
        sim.step()
        n += 1
    el = time.perf_counter() - t0
    gm = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=device())
    st = swe.State(gm, fixed, precision=swe.FP32 if precision == "fp32" else swe.FP64)
    for _ in range(n):
        st.step()
    errs, _ = errors(st.read(), sim)
    st.close()
    gm.close()
    return dict(steps=n, seconds=el, prep=prep, rate=sc.n_cells * n / el, errors=errs)


def bench_batched(n_members=64, rounds=8, k=16):
    """Batched ensemble: members of the lake generator (jittered-lattice mesh
    for generation speed) with log-uniform sizes, each fed by its own
    hydrograph, stepped together by one persistent kernel per step; against
    the same members stepped one after another through the single-solve
    API for the same number of steps."""
    import torch
    import swe_inputs as S
    from gpu_util import cached, device
    from paper_2102_12862_amd import swe
    sizes = S.ensemble_sizes(n_members)
    members = [cached("ens_lattice", S.ensemble_member, k, int(n), mesh="lattice") for k, n in enumerate(sizes)]
    dev = device()
    meshes = [swe.Mesh(m.nodes, m.tri, m.bnd_seg, m.bnd_tag, device=dev) for m in members]
    total = sum(m.n_cells for m in members)
    # batched
    states = [swe.State(me, m, precision=swe.FP32) for me, m in zip(meshes, members)]
    batch = swe.Batch(precision=swe.FP32, device=dev)
    for st in states:
        batch.add(st, 1e9)
    batch.step(k)  # warm-up (capture)
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record(dev.stream)
    for _ in range(rounds):
        batch.launch(k)
    e1.record(dev.stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    batch.close()
    for st in states:
        st.close()
    # one after another
    states = [swe.State(me, m, precision=swe.FP32, steps_per_graph=k) for me, m in zip(meshes, members)]
    for st in states:
        st.launch_steps(k)
    torch.cuda.synchronize()
    e0.record(dev.stream)
    for _ in range(rounds):
        for st in states:
            st.launch_steps(k)
    e1.record(dev.stream)
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1)
    for st in states:
        st.close()
    for me in meshes:
        me.close()
    steps = rounds * k
    return {"members": n_members, "cells": int(total), "steps_each": steps,
            "batched_cell_updates_per_s": total * steps / (ms_b * 1e-3),
            "sequential_cell_updates_per_s": total * steps / (ms_s * 1e-3),
            "speedup": ms_s / ms_b}


def bench_serving(n_requests=24, rate=4.0):
    """Served Poisson trace of valley-flood requests (domain scaled so the
    cell size stays the valley's), continuous batching with footprint
    admission; against the same trace served one request at a time."""
    import swe_inputs as S
    from gpu_util import cached, device
    from paper_2102_12862_amd import serve, swe
    arrive, sizes, horizon = S.serving_trace(n_requests=n_requests, rate=rate, n_lo=1e4, n_hi=2e6,
                                             h_lo=60.0, h_hi=1800.0)
    scen = [cached("req", S.serving_request, i, int(n), float(h)) for i, (n, h) in enumerate(zip(sizes, horizon))]

    def reqs():
        return [serve.Request(i, float(a), (lambda sc=scen[i]: sc), float(horizon[i])) for i, a in enumerate(arrive)]

    dev = device()
    srv = serve.Server(precision=swe.FP32, budget_bytes=2 << 30, steps_per_round=32, device=dev,
                       keep_results=False)
    r1 = reqs()
    t0 = time.perf_counter()
    srv.serve(r1)
    wall = time.perf_counter() - t0
    srv.close()
    s_batched = serve.summarize(r1, wall)
    r2 = reqs()
    t0 = time.perf_counter()
    serve.serve_sequential(r2, precision=swe.FP32, device=dev)
    wall2 = time.perf_counter() - t0
    s_seq = serve.summarize(r2, wall2)
    return {"requests": n_requests, "rate_per_s": rate, "cells_range": [1e4, 2e6], "horizon_s": [60, 1800],
            "served": s_batched, "one_at_a_time": s_seq}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="valley_wet")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--tile", type=int, default=0, choices=(0, 128, 256, 512),
                    help="cells per tile (block size) of the step kernel; 0: autotuned")
    ap.add_argument("--morpho", action="store_true", help="carry the Exner module (MPM closure)")
    ap.add_argument("--species", type=int, default=0, choices=range(0, 6),
                    help="passive species carried by the step (0: the hydrodynamic step alone)")
    ap.add_argument("--kernel-digest", action="store_true", help="print the digest of the kernel sources and exit")
    args = ap.parse_args()
    if args.kernel_digest:
        print(kernel_digest())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path is one device's share of the mesh; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        # a plain elementwise kernel that reads and writes a known number of
        # bytes once each, to scale the HBM byte counters
        n = (args.copy_calibration_mib << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration_mib} MiB read + written per launch (3 launches)")
        del x, y
    log(f"[bench] generating {args.workload}")
    t0 = time.perf_counter()
    sc = make_workload(args.workload)
    log(f"[bench] {sc.name}: {sc.n_cells} cells ({time.perf_counter() - t0:.1f}s)")
    r = time_gpu(sc, args.precision, args.steps, args.warmup, autotune=not args.no_autotune, species=args.species,
                 tile=args.tile, morpho=args.morpho)
    N = sc.n_cells
    value = r["rate"]
    bytes_per_cell = ALGO_BYTES[args.precision] + args.species * SPECIES_BYTES[args.precision]
    achieved = bytes_per_cell * N / (r["ms_step"] * 1e-3) / 1e9
    tile = r["tune"][0] if r["tune"] else (args.tile or 256)
    traffic = measured_traffic(sc.name, args.precision, tile, args.species, args.morpho)
    tname = "float" if args.precision == "fp32" else "double"
    kname = (f"k_step_morpho<{tname}, 256>" if args.morpho else
             f"k_step_species<{tname}, 256, {args.species}, false>" if args.species
             else f"k_step<{tname}, {tile}, false, false, false>")
    log(f"[bench] gpu {args.precision}: {r['ms_step'] * 1e3:.1f} us/step, {value:.3e} cell-updates/s, "
        f"{achieved:.0f} GB/s algorithmic, tune {r['tune']}")
    variants = {}
    if not args.no_variants:
        other = "fp64" if args.precision == "fp32" else "fp32"
        o = time_gpu(sc, other, max(50, args.steps // 5), 10)
        variants[f"{sc.name}_{other}"] = {"cell_updates_per_s": o["rate"], "us_per_step": o["ms_step"] * 1e3,
                                          "roofline_frac": ALGO_BYTES[other] * N / (o["ms_step"] * 1e-3) / 1e9
                                          / HBM_PEAK_GBS, "block_cpt": o["tune"],
                                          "traffic": measured_traffic(sc.name, other, o["tune"][0])}
        log(f"[bench] {other}: {o['ms_step'] * 1e3:.1f} us/step")
        lake = make_workload("lake")
        for p in ("fp32", "fp64"):
            lr = time_gpu(lake, p, 500, 50)
            variants[f"{lake.name}_{p}"] = {"cell_updates_per_s": lr["rate"], "us_per_step": lr["ms_step"] * 1e3,
                                           "note": "working set fits the 256 MB Infinity Cache"}
            log(f"[bench] lake {p}: {lr['ms_step'] * 1e3:.1f} us/step")
        if not (args.species or args.morpho):
            mr = time_gpu(sc, args.precision, max(50, args.steps // 5), 10, morpho=True)
            variants[f"{sc.name}_{args.precision}_morpho"] = {
                "cell_updates_per_s": mr["rate"], "us_per_step": mr["ms_step"] * 1e3,
                "algorithmic_bytes_per_cell": ALGO_BYTES[args.precision],
                "roofline_frac": ALGO_BYTES[args.precision] * N / (mr["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
            log(f"[bench] Exner (MPM): {mr['ms_step'] * 1e3:.1f} us/step")
        for ns in ((2, 5) if not (args.species or args.morpho) else ()):
            sr = time_gpu(sc, args.precision, max(50, args.steps // 5), 10, species=ns)
            b = ALGO_BYTES[args.precision] + ns * SPECIES_BYTES[args.precision]
            variants[f"{sc.name}_{args.precision}_species{ns}"] = {
                "cell_updates_per_s": sr["rate"], "us_per_step": sr["ms_step"] * 1e3,
                "algorithmic_bytes_per_cell": b,
                "roofline_frac": b * N / (sr["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
            log(f"[bench] {ns} species: {sr['ms_step'] * 1e3:.1f} us/step")
        log("[bench] batched ensemble")
        variants["batched_ensemble_fp32"] = bench_batched()
        log(f"[bench] batched: {variants['batched_ensemble_fp32']}")
        log("[bench] serving trace")
        variants["served_trace_fp32"] = bench_serving()
        log(f"[bench] serving: {variants['served_trace_fp32']}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle sample")
        o = time_oracle(sc, precision=args.precision)
        cpu = {"value": o["rate"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"{o['steps']} FP64 steps of the same {N}-cell workload, time step fixed at half "
                         f"the initial CFL step ({o['seconds']:.1f}s, serial C)",
               "gpu_error_vs_oracle": o["errors"]}
        log(f"[bench] oracle {o['rate']:.3e} cell-updates/s; gpu errors {o['errors']}")
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": sc.name, "cells": N, "precision": args.precision,
                   "state": "fully wet snapshot" if "wet" in args.workload else "as generated",
                   "block_size_cells_per_thread": r["tune"], "species": args.species, "morpho": args.morpho},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_cell": bytes_per_cell,
                     "algorithmic_bytes_per_launch": bytes_per_cell * N,
                     "kernel": kname},
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
