"""Benchmark of the shallow-water step on one MI355X.

Headline workload: the valley flood (4M-triangle Delaunay mesh of a jittered
lattice over a 20 km x 4 km synthetic DEM with a meandering channel), fully
wet snapshot (1 m of water moving at 0.5 m/s, so every cell does the whole
step), FP32 state with FP64 depth tests / dt / mass, stepped through hipGraph
launches of the C-ABI library.  A step is one full pass of the method over
every cell: reconstruction, HLLC, update, friction, positivity and the
device-side CFL reduction.

Timing protocol (every timed figure): W untimed warm-up steps, the hipGraphs
of the timed chunks captured before the timed region, then exactly K steps as
a few equal graph launches with HIP events between them on the library's
stream; the value is K steps over their total time, and the chunks' median is
reported beside it.

Prints one JSON line: cell-updates/s, the roofline object of the step kernel
(algorithmic bytes per cell-update x cells / time per step), the FP64 oracle
timed on a bounded sample on the host's cores (all of them, and one), and
under "variants" the same measurements for FP64, the valley flood run from its
dry start to the end of its hydrograph (t = 3600 s), the 200k-cell lake at
rest, the passive-species and Exner steps, a batched ensemble against the same
members solved one after another, and a served Poisson request trace at
several arrival rates against one-at-a-time serving.  Every variant carries
its max and L1 errors against the oracle on a sample.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
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
VALLEY_T_END = 3600.0
AUTOTUNE_STEPS = 20  # steps per tile size and round of the autotuner


# HBM traffic of the step kernel, measured with the FETCH_SIZE and WRITE_SIZE
# counters (each scaled by what it reads for a plain copy of known size); it
# is reported only while the kernel sources still hash to the digest recorded
# with the measurement
def traffic_profile(precision, species, morpho=False, batched=False):
    if batched:
        return os.path.join(ROOT, "profiles", f"k_step_batched_{precision}_ensemble64_hbm_traffic.md")
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


def measured_traffic(workload, precision, tile, species=0, morpho=False, batched=False):
    """Bytes per step-kernel launch from the committed counter profile, or
    None when it was taken on other kernel sources or another configuration."""
    try:
        with open(traffic_profile(precision, species, morpho, batched)) as fh:
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


def valley_dry():
    import swe_inputs as S
    from gpu_util import cached
    return cached("valley", S.valley_flood, n_cells=4_000_000)


def make_workload(name):
    import swe_inputs as S
    from gpu_util import cached
    if name == "valley_wet":
        return S.wet_snapshot(valley_dry())
    if name in ("valley_dry", "valley_tend"):
        return valley_dry()
    if name == "lake":
        return cached("lake", S.lake_at_rest, n_cells=200_000)
    raise SystemExit(f"unknown workload {name}")


def host_threads():
    """Cores this process may use: its CPU affinity, capped by OMP_NUM_THREADS
    when that is set (a shared host's share)."""
    n = len(os.sched_getaffinity(0))
    try:
        return max(1, min(n, int(os.environ["OMP_NUM_THREADS"])))
    except (KeyError, ValueError):
        return n


def host_info():
    info = {"nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count(), "threads_used": host_threads()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def species_phi0(sc, ns):
    """Initial concentrations of ns species: a front across the domain at
    the median centroid x, then uniform backgrounds."""
    cx = sc.centroids()[:, 0]
    rows = [np.where(cx < np.median(cx), 1.0, 0.0)] + [np.full(sc.n_cells, 0.1 * (k + 1)) for k in range(ns - 1)]
    return np.stack(rows[:ns])


def n_chunks(steps):
    return next((c for c in (5, 4, 3) if steps % c == 0), 1)


def timed_steps(st, dev, steps, warmup):
    """W untimed warm-up steps, then exactly `steps` steps as equal hipGraph
    launches (captured before the timed region) with HIP events between them
    on the library's stream.  Returns the total and per-chunk times."""
    import torch
    nch = n_chunks(steps)
    per = steps // nch
    st.prepare_graphs(per)
    st.launch_steps(warmup)
    st.sync()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nch + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(dev.stream)
    for c in range(nch):
        st.launch_steps(per)
        ev[c + 1].record(dev.stream)
    st.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    chunk_ms = [ev[c].elapsed_time(ev[c + 1]) for c in range(nch)]
    ms = ev[0].elapsed_time(ev[nch])
    return dict(ms=ms, wall=wall, ms_step=ms / steps, chunks=nch, steps_per_chunk=per,
                chunk_us_per_step=[1e3 * c / per for c in chunk_ms],
                median_us_per_step=float(np.median([1e3 * c / per for c in chunk_ms])))


def gpu_state(sc, precision, tile=0, species=0, morpho=False):
    from paper_2102_12862_amd import swe
    from gpu_util import device
    mesh = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=device())
    p = swe.FP32 if precision == "fp32" else swe.FP64
    st = swe.State(mesh, sc, precision=p, block_size=tile)
    if species:
        st.set_scalars(species_phi0(sc, species))
    if morpho:
        import swe_inputs as S
        st.set_morpho(S.Morpho("mpm"))
    return mesh, st


def time_gpu(sc, precision, steps, warmup, autotune=True, species=0, tile=0, morpho=False, state=None):
    """Time per step over `steps` graph-launched steps (timed_steps)."""
    from gpu_util import device
    mesh, st = state if state is not None else gpu_state(sc, precision, tile, species, morpho)
    tune = st.autotune(k=AUTOTUNE_STEPS) if (autotune and not tile and not (species or morpho)) else None
    r = timed_steps(st, device(), steps, warmup)
    st.close()
    mesh.close()
    r.update(tile=tune or tile or 256, autotuned=tune is not None, rate=sc.n_cells * steps / (r["ms"] * 1e-3))
    return r


def fixed_dt(sc, om, frac=0.5):
    """The scenario with its time step fixed at `frac` of the oracle's first
    CFL step: FP32 and FP64 states of a trajectory then step with the same
    dt (their CFL steps differ by rounding, and a different dt is not an
    error of the step)."""
    import oracle
    import swe_inputs as S
    fixed = S.Scenario(**{**sc.__dict__})
    fixed.dt_max = frac * oracle.Sim(sc, mesh=om).next_dt()
    return fixed


def error_sample(sc, precision, steps, om=None, species=0, morpho=False, tile=0):
    """Max and L1 errors in h, qx, qy (and the species' specific masses) of
    `steps` GPU steps against as many oracle steps from the same initial
    state, with the time step fixed (fixed_dt)."""
    import oracle
    from gpu_util import errors
    om = om or oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, omp=True)
    fixed = fixed_dt(sc, om)
    if species:
        fixed.phi0 = species_phi0(sc, species)
    if morpho:
        import swe_inputs as S
        fixed.morpho = S.Morpho("mpm")
    sim = oracle.Sim(fixed, mesh=om)
    mesh, st = gpu_state(fixed, precision, tile)  # the scenario carries the species and the Exner module
    for _ in range(steps):
        st.step()
    sim.run_steps(steps)
    errs, _ = errors(st.read(), sim)
    if species:
        q, qr = st.scalars(), sim.scalars()
        for c in range(species):
            s = max(np.abs(qr[c]).max(), 1e-300)
            errs[f"max_q{c + 1}"] = float(np.abs(q[c] - qr[c]).max() / s)
    st.close()
    mesh.close()
    return {"steps": steps, **{k: float(v) for k, v in errs.items()}}


def time_oracle(sc, om_serial, om_omp, budget_s=10.0, max_steps=200):
    """The FP64 oracle on a bounded sample of the workload (steps with the
    time step fixed at half the initial CFL step): the serial build on one
    core and the OpenMP build of the same source on every core of the host."""
    import oracle
    out = {}
    fixed = fixed_dt(sc, om_serial)
    for name, om in (("serial", om_serial), ("openmp", om_omp)):
        threads = oracle.threads(host_threads()) if name == "openmp" else 1
        sim = oracle.Sim(fixed, mesh=om)
        sim.step()  # warm-up (first touch of the state arrays)
        n = 0
        t0 = time.perf_counter()
        while n < max_steps and time.perf_counter() - t0 < budget_s:
            sim.step()
            n += 1
        el = time.perf_counter() - t0
        out[name] = {"rate": sc.n_cells * n / el, "steps": n, "seconds": el, "threads": threads}
    return out


def valley_to_t_end(sc, precision, steps, warmup, tile=0):
    """The valley flood as configured: dry start, inflow hydrograph 50 ->
    2000 m^3/s over one hour, run to t = 3600 s on the GPU; then the step
    timed on the state at t_end.  Reports the run's step count and time, its
    volume balance, the delivered inflow volume against the hydrograph's
    integral, and the wet fraction."""
    from paper_2102_12862_amd import swe
    from gpu_util import device
    mesh, st = gpu_state(sc, precision, tile)
    m0 = st.mass()
    t0 = time.perf_counter()
    n = st.run_until(VALLEY_T_END)
    run_wall = time.perf_counter() - t0
    m1 = st.mass()
    got = st.read()
    q = sc.bcs[0]
    delivered = -st.boundary_flux(q.tag)  # volume that entered through the inflow edges
    tune = st.autotune(k=AUTOTUNE_STEPS) if not tile else None
    # every later step is capped at t_end: step on past it for the timing
    r = timed_steps_after(st, device(), steps, warmup)
    st.close()
    mesh.close()
    inflow = float(sum(0.5 * (q.Q[i] + q.Q[i + 1]) * (q.t[i + 1] - q.t[i]) for i in range(len(q.t) - 1))) \
        if VALLEY_T_END >= q.t[-1] else None
    wet = float((got["h"] > sc.h_min).mean())
    resid = (m1["mass"] - m0["mass"] + m1["bnd_flux"] - m1["clipped"]) / max(m1["mass"], 1e-300)
    r.update(tile=tune or tile or 256, rate=sc.n_cells * steps / (r["ms"] * 1e-3), run_steps=int(n),
             run_wall_s=run_wall, run_mean_us_per_step=1e6 * run_wall / max(n, 1), t=got["t"],
             wet_fraction=wet, volume=m1["mass"], clipped=m1["clipped"], balance_residual_rel=resid,
             bnd_flux=m1["bnd_flux"], inflow_volume_hydrograph=inflow, inflow_volume_delivered=delivered,
             delivered_over_hydrograph=(delivered / inflow) if inflow else None)
    return r


def timed_steps_after(st, dev, steps, warmup):
    st.launch_steps(0, t_end=float("inf"))  # lifts the end-time cap
    return timed_steps(st, dev, steps, warmup)


def bench_batched(n_members=64, rounds=8, k=16, t_end=1800.0, horizon=True):
    """Batched ensemble: members of the lake generator (its 28-degree
    Poisson-disk Delaunay meshes) with log-uniform sizes, each fed by its own
    hydrograph, stepped together by one persistent kernel per step (tile
    chosen by the batched autotuner); against the same members stepped one
    after another through the single-solve API for the same number of steps.
    Then the whole ensemble run on to its horizon t_end (members finish at
    their own step counts), with the errors of the smallest member against
    the oracle at t_end (horizon=False skips that part, so that a profile of
    the run holds the timed steps only)."""
    import torch
    import oracle
    import swe_inputs as S
    from gpu_util import cached, device, errors
    from paper_2102_12862_amd import swe
    sizes = S.ensemble_sizes(n_members)
    members = parallel_generate([("ens", S.ensemble_member, (k, int(n)), {}) for k, n in enumerate(sizes)],
                                workers=16)
    dev = device()
    meshes = [swe.Mesh(m.nodes, m.tri, m.bnd_seg, m.bnd_tag, device=dev) for m in members]
    total = sum(m.n_cells for m in members)
    steps = rounds * k
    # batched
    states = [swe.State(me, m, precision=swe.FP32) for me, m in zip(meshes, members)]
    batch = swe.Batch(precision=swe.FP32, device=dev)
    for st in states:
        batch.add(st, t_end)
    tile = batch.autotune(8)
    batch.step(k)  # warm-up (capture)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(rounds + 1)]
    torch.cuda.synchronize()
    ev[0].record(dev.stream)
    for i in range(rounds):
        batch.launch(k)
        ev[i + 1].record(dev.stream)
    torch.cuda.synchronize()
    ms_b = ev[0].elapsed_time(ev[rounds])
    chunk = [1e3 * ev[i].elapsed_time(ev[i + 1]) / k for i in range(rounds)]
    # on to the horizon
    horizon_out, errs_out = None, None
    if horizon:
        t0 = time.perf_counter()
        while batch.step(64):
            pass
        run_wall = time.perf_counter() - t0
        member_steps = [int(st.mass()["steps"]) for st in states]
        run_updates = sum(n * m.n_cells for n, m in zip(member_steps, members))
        small = int(np.argmin([m.n_cells for m in members]))
        got = states[small].read()
        sim = oracle.Sim(members[small], omp=True)
        sim.run_until(got["t"])
        errs, _ = errors(got, sim)
        horizon_out = {"t_end": t_end, "wall_s": run_wall, "member_steps_min": min(member_steps),
                       "member_steps_max": max(member_steps), "cell_updates": run_updates,
                       "cell_updates_per_s": run_updates / run_wall}
        errs_out = {"member_cells": members[small].n_cells, "t": got["t"], **{kk: float(v) for kk, v in errs.items()}}
    batch.close()
    for st in states:
        st.close()
    log(f"[bench] batched: {1e3 * ms_b / steps:.1f} us per step of all members; members one after another")
    # one after another
    states = [swe.State(me, m, precision=swe.FP32, steps_per_graph=k) for me, m in zip(meshes, members)]
    for st in states:
        st.prepare_graphs(k)
        st.launch_steps(k)
    torch.cuda.synchronize()
    ev[0].record(dev.stream)
    for _ in range(rounds):
        for st in states:
            st.launch_steps(k)
    ev[1].record(dev.stream)
    torch.cuda.synchronize()
    ms_s = ev[0].elapsed_time(ev[1])
    for st in states:
        st.close()
    for me in meshes:
        me.close()
    rate_b = total * steps / (ms_b * 1e-3)
    achieved = ALGO_BYTES["fp32"] * rate_b / 1e9
    return {"members": n_members, "cells": int(total), "steps_each": steps, "tile": tile,
            "batched_cell_updates_per_s": rate_b, "median_us_per_step": float(np.median(chunk)),
            "sequential_cell_updates_per_s": total * steps / (ms_s * 1e-3), "speedup": ms_s / ms_b,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_cell": ALGO_BYTES["fp32"],
                         "traffic": measured_traffic(f"batched_ensemble_{n_members}", "fp32", tile, batched=True),
                         "kernel": f"k_step_batched<float, {tile}, false>"},
            "run_to_horizon": horizon_out, "errors_vs_oracle": errs_out}


def _gen(args):
    name, fn, a, kw = args
    from gpu_util import cached
    return cached(name, fn, *a, **kw)


def parallel_generate(jobs, workers=8):
    """Scenario generation in worker processes (deterministic and cached on
    disk, so the order of completion does not matter)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=max(1, min(workers, host_threads(), len(jobs))),
                                mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_gen, jobs))


def bench_serving(rates=(4.0, 16.0, 64.0), n_requests=48, n_pool=12, long_trace=(64.0, 512)):
    """Served Poisson traces of valley-flood requests on a cached pool of
    prepared domains (each pool domain scaled so the cell size stays the
    valley's; a request takes the pool domain nearest its log-uniform size,
    with its own horizon), continuous batching with footprint admission;
    against the same trace served one request at a time, at each arrival
    rate; then one long trace (rate, requests) the same way.  Errors of one
    served result against the oracle."""
    import oracle
    import swe_inputs as S
    from gpu_util import device, errors
    from paper_2102_12862_amd import serve, swe
    sizes = S.serving_pool(n_pool)
    pool = parallel_generate([("req", S.serving_request, (k, int(n), 1800.0), {}) for k, n in enumerate(sizes)])
    dev = device()
    meshes = [swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=dev) for sc in pool]
    out = {"pool_cells": [int(sc.n_cells) for sc in pool], "requests_per_rate": n_requests,
           "cells_range": [1e4, 2e6], "horizon_s": [60, 1800], "rates": {}}
    sample = None
    traces = [(rate, n_requests) for rate in rates] + ([tuple(long_trace)] if long_trace and long_trace[1] else [])
    for rate, nreq in traces:
        arrive, want, horizon = S.serving_trace(n_requests=nreq, rate=rate, n_lo=1e4, n_hi=2e6,
                                                h_lo=60.0, h_hi=1800.0)
        pick = [int(np.argmin(np.abs(np.log(sizes) - np.log(n)))) for n in want]

        def reqs():
            return [serve.Request(i, float(a), (lambda k=pick[i], h=float(horizon[i]), i=i: S.pool_request(pool[k], i, h)),
                                  float(horizon[i]), mesh=meshes[pick[i]])
                    for i, a in enumerate(arrive)]

        srv = serve.Server(precision=swe.FP32, budget_bytes=2 << 30, steps_per_round=32, device=dev,
                           keep_results=sample is None)
        r1 = reqs()
        t0 = time.perf_counter()
        srv.serve(r1)
        wall = time.perf_counter() - t0
        srv.close()
        if sample is None:
            i = int(np.argmin([r.cells if r.error is None else 1 << 62 for r in r1]))
            sample = (r1[i], S.pool_request(pool[pick[i]], i, float(horizon[i])))
        r2 = reqs()
        t0 = time.perf_counter()
        serve.serve_sequential(r2, precision=swe.FP32, device=dev)
        wall2 = time.perf_counter() - t0
        key = f"{rate:g}" if nreq == n_requests else f"{rate:g}x{nreq}"
        out["rates"][key] = {"served": serve.summarize(r1, wall), "one_at_a_time": serve.summarize(r2, wall2)}
        log(f"[bench] serving {nreq} requests at {rate:g}/s: {out['rates'][key]}")
    for me in meshes:
        me.close()
    r, sc = sample
    sim = oracle.Sim(sc, omp=True)
    sim.run_until(sc.t_end)
    errs, _ = errors(r.result, sim)
    out["errors_vs_oracle"] = {"request_cells": sc.n_cells, "horizon_s": sc.t_end,
                               **{k: float(v) for k, v in errs.items()}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="valley_wet", choices=["valley_wet", "valley_tend", "lake"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated variants to run (default: all)")
    ap.add_argument("--serving-requests", type=int, default=48, help="requests per arrival rate")
    ap.add_argument("--serving-long", type=int, default=512,
                    help="requests of the long served trace at 64 per second (0: none)")
    ap.add_argument("--no-batched-horizon", action="store_true",
                    help="skip running the batched ensemble on to its horizon (for profiles of the timed steps)")
    ap.add_argument("--batched-rounds", type=int, default=8,
                    help="timed rounds of 16 steps of the batched ensemble (and of its one-after-another baseline)")
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
    only = set(filter(None, args.only.split(",")))

    def want(name):
        return not args.no_variants and (not only or name in only)

    log(f"[bench] generating {args.workload}")
    t0 = time.perf_counter()
    sc = make_workload(args.workload)
    log(f"[bench] {sc.name}: {sc.n_cells} cells ({time.perf_counter() - t0:.1f}s)")
    N = sc.n_cells
    if args.workload == "valley_tend":
        r = valley_to_t_end(sc, args.precision, args.steps, args.warmup, tile=args.tile)
    else:
        r = time_gpu(sc, args.precision, args.steps, args.warmup, autotune=not args.no_autotune,
                     species=args.species, tile=args.tile, morpho=args.morpho)
    value = r["rate"]
    bytes_per_cell = ALGO_BYTES[args.precision] + args.species * SPECIES_BYTES[args.precision]
    achieved = bytes_per_cell * N / (r["ms_step"] * 1e-3) / 1e9
    tile = r["tile"]
    traffic = measured_traffic(sc.name, args.precision, tile, args.species, args.morpho)
    tname = "float" if args.precision == "fp32" else "double"
    kname = (f"k_step_morpho<{tname}, 256>" if args.morpho else
             f"k_step_species<{tname}, 256, {args.species}, false>" if args.species
             else f"k_step<{tname}, {tile}, false, false, false>")
    log(f"[bench] gpu {args.precision}: {r['ms_step'] * 1e3:.1f} us/step (median chunk "
        f"{r['median_us_per_step']:.1f}), {value:.3e} cell-updates/s, {achieved:.0f} GB/s algorithmic, tile {tile}")
    import oracle
    om_serial = om_omp = None
    if args.workload != "lake" and (want("errors") or not args.no_cpu_baseline or want("fp64")
                                    or want("species") or want("morpho")):
        om_serial = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
        om_omp = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, omp=True)
        oracle.threads(host_threads())
    variants = {}
    wet = make_workload("valley_wet") if args.workload == "valley_tend" else sc
    other = "fp64" if args.precision == "fp32" else "fp32"
    if want("fp64") and args.workload != "lake":
        o = time_gpu(wet, other, max(60, args.steps // 5), 10)
        variants[f"{wet.name}_{other}"] = {
            "cell_updates_per_s": o["rate"], "us_per_step": o["ms_step"] * 1e3,
            "median_us_per_step": o["median_us_per_step"], "tile": o["tile"],
            "roofline_frac": ALGO_BYTES[other] * N / (o["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": measured_traffic(wet.name, other, o["tile"]),
            "errors_vs_oracle": error_sample(wet, other, 3, om_omp, tile=o["tile"])}
        log(f"[bench] {other}: {variants[f'{wet.name}_{other}']}")
    if want("prep"):
        # mesh preparation (edge table, orientation, FP64 geometry, Hilbert
        # order, boundary slots, tile edge lists) and its upload, once per mesh
        from paper_2102_12862_amd import swe
        prep = []
        for _ in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            m = swe.Mesh(wet.nodes, wet.tri, wet.bnd_seg, wet.bnd_tag, device=_dev())
            torch.cuda.synchronize()
            prep.append(time.perf_counter() - t1)
            m.close()
        variants["mesh_prep"] = {"cells": int(N), "seconds": min(prep), "host_threads": 1}
        log(f"[bench] mesh preparation: {variants['mesh_prep']}")
    if want("tend") and args.workload == "valley_wet":
        dry = valley_dry()
        for p in ("fp32", "fp64"):
            tr = valley_to_t_end(dry, p, max(60, args.steps // 5), 10)
            b = ALGO_BYTES[p]
            variants[f"{dry.name}_t3600_{p}"] = {
                **{k: v for k, v in tr.items() if k not in ("ms", "wall")},
                "cell_updates_per_s": tr["rate"], "us_per_step": tr["ms_step"] * 1e3,
                "roofline_frac": b * N / (tr["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
            log(f"[bench] valley to t=3600 s {p}: {variants[f'{dry.name}_t3600_{p}']}")
    if want("lake"):
        lake = make_workload("lake")
        for p in ("fp32", "fp64"):
            mesh, st = gpu_state(lake, p)
            H0 = st.read()["H"]
            tl = st.autotune(k=AUTOTUNE_STEPS)
            lr = timed_steps(st, _dev(), 500, 50)
            got = st.read()
            rest = {"steps": int(st.mass()["steps"]),
                    "max_abs_q": float(max(np.abs(got["qx"]).max(), np.abs(got["qy"]).max())),
                    "surface_bitwise_unchanged": bool(np.array_equal(got["H"], H0))}
            st.close()
            mesh.close()
            variants[f"{lake.name}_{p}"] = {"cell_updates_per_s": lake.n_cells * 500 / (lr["ms"] * 1e-3),
                                           "us_per_step": lr["ms_step"] * 1e3, "tile": tl,
                                           "median_us_per_step": lr["median_us_per_step"],
                                           "lake_at_rest": rest,
                                           "note": "working set fits the 256 MB Infinity Cache"}
            log(f"[bench] lake {p}: {variants[f'{lake.name}_{p}']}")
    if args.workload == "valley_wet" and not (args.species or args.morpho):
        if want("morpho"):
            mr = time_gpu(wet, args.precision, max(60, args.steps // 5), 10, morpho=True)
            variants[f"{wet.name}_{args.precision}_morpho"] = {
                "cell_updates_per_s": mr["rate"], "us_per_step": mr["ms_step"] * 1e3,
                "median_us_per_step": mr["median_us_per_step"], "tile": 256,
                "algorithmic_bytes_per_cell": ALGO_BYTES[args.precision],
                "roofline_frac": ALGO_BYTES[args.precision] * N / (mr["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "errors_vs_oracle": error_sample(wet, args.precision, 3, om_serial, morpho=True)}
            log(f"[bench] Exner (MPM): {variants[f'{wet.name}_{args.precision}_morpho']}")
        if want("species"):
            for ns in (2, 5):
                sr = time_gpu(wet, args.precision, max(60, args.steps // 5), 10, species=ns)
                b = ALGO_BYTES[args.precision] + ns * SPECIES_BYTES[args.precision]
                variants[f"{wet.name}_{args.precision}_species{ns}"] = {
                    "cell_updates_per_s": sr["rate"], "us_per_step": sr["ms_step"] * 1e3,
                    "median_us_per_step": sr["median_us_per_step"], "tile": 256,
                    "algorithmic_bytes_per_cell": b,
                    "roofline_frac": b * N / (sr["ms_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "errors_vs_oracle": error_sample(wet, args.precision, 3, om_serial, species=ns)}
                log(f"[bench] {ns} species: {variants[f'{wet.name}_{args.precision}_species{ns}']}")
    if want("batched"):
        log("[bench] batched ensemble")
        variants["batched_ensemble_fp32"] = bench_batched(rounds=args.batched_rounds,
                                                          horizon=not args.no_batched_horizon)
        log(f"[bench] batched: {variants['batched_ensemble_fp32']}")
    if want("serving"):
        log("[bench] serving traces")
        variants["served_traces_fp32"] = bench_serving(n_requests=args.serving_requests,
                                                       long_trace=(64.0, args.serving_long))
    errs = None
    if want("errors") and args.workload == "valley_wet":
        errs = error_sample(wet, args.precision, 20, om_omp, tile=tile, species=args.species, morpho=args.morpho)
        log(f"[bench] errors vs oracle: {errs}")
    cpu = None
    if not args.no_cpu_baseline and om_serial is not None:
        log("[bench] oracle timing")
        o = time_oracle(wet, om_serial, om_omp)
        lake = make_workload("lake")
        lom, lomp = oracle.Mesh(lake.nodes, lake.tri), oracle.Mesh(lake.nodes, lake.tri, omp=True)
        ol = time_oracle(lake, lom, lomp, budget_s=4.0)
        cpu = {"value": o["openmp"]["rate"], "unit": "cell-updates/s", "cores": o["openmp"]["threads"],
               "kind": "oracle",
               "sample": f"{o['openmp']['steps']} FP64 steps of the same {N}-cell workload (time step fixed "
                         f"at half the initial CFL step) with the OpenMP build of the oracle on every host core "
                         f"({o['openmp']['seconds']:.1f} s)",
               "serial_1core": {"value": o["serial"]["rate"], "steps": o["serial"]["steps"],
                                "seconds": o["serial"]["seconds"]},
               "lake_200k": {"openmp": ol["openmp"], "serial": ol["serial"]},
               "host": host_info()}
        log(f"[bench] oracle: {cpu}")
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
        "config": {"workload": sc.name if args.workload != "valley_tend" else sc.name + "_t3600",
                   "cells": N, "precision": args.precision,
                   "state": {"valley_wet": "fully wet snapshot", "valley_tend": "state at t = 3600 s of the dry start",
                             "lake": "lake at rest"}[args.workload],
                   "tile": tile, "autotuned": r.get("autotuned", False), "species": args.species,
                   "morpho": args.morpho, "timing": {"chunks": r["chunks"], "steps_per_chunk": r["steps_per_chunk"],
                                                      "chunk_us_per_step": r["chunk_us_per_step"],
                                                      "median_us_per_step": r["median_us_per_step"]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_cell": bytes_per_cell,
                     "algorithmic_bytes_per_launch": bytes_per_cell * N,
                     "kernel": kname},
        "errors_vs_oracle": errs,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


def _dev():
    from gpu_util import device
    return device()


if __name__ == "__main__":
    main()
