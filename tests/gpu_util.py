"""Helpers shared by the GPU tests: run a scenario through the C ABI and
through the oracle, and compare them."""
from __future__ import annotations

import functools
import os
import pickle

import numpy as np

import swe_inputs as S

CACHE = os.environ.get("SWE_MESH_CACHE", "/tmp/swe_mesh_cache")


def cached(name, fn, *args, **kw):
    """Scenario generation is deterministic; large meshes are cached on disk
    for the duration of a run (files written by this process only)."""
    os.makedirs(CACHE, exist_ok=True)
    key = name + "_" + "_".join(f"{a}" for a in args) + "_" + "_".join(f"{k}{v}" for k, v in sorted(kw.items()))
    path = os.path.join(CACHE, key + ".pkl")
    if os.path.exists(path):
        with open(path, "rb") as f:
            return pickle.load(f)
    sc = fn(*args, **kw)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "wb") as f:
        pickle.dump(sc, f)
    os.replace(tmp, path)
    return sc


@functools.lru_cache(maxsize=None)
def device():
    from paper_2102_12862_amd import swe
    return swe.TorchDevice()


def gpu_state(sc, precision, mesh=None, **params):
    from paper_2102_12862_amd import swe
    renumber = params.pop("renumber", True)
    if mesh is None:
        mesh = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=device(), renumber=renumber)
    return swe.State(mesh, sc, precision=precision, **params)


def rel_err(got, ref, floor=1e-300):
    """max |got - ref| / max |ref| (norm-relative, as stated for parity)."""
    d = np.abs(got - ref).max()
    s = np.abs(ref).max()
    if s < floor:
        return float(d)
    return float(d / s)


def l1_rel(got, ref, w):
    return float((np.abs(got - ref) * w).sum() / max((np.abs(ref) * w).sum(), 1e-300))


def errors(got, sim):
    """Norm-relative max and area-weighted L1 errors of h, qx, qy (and the
    max error of H) of a GPU read-out against the oracle."""
    H, qx, qy, t = sim.state()
    geo = sim.mesh.geometry()
    zb, area = sim.bed(), geo["area"]   # the bed as it stands (it moves under morphodynamics)
    ref = dict(H=H, h=H - zb, qx=qx, qy=qy)
    out = {}
    for f in ("H", "h", "qx", "qy"):
        out["max_" + f] = rel_err(got[f], ref[f])
        if f != "H":
            out["l1_" + f] = l1_rel(got[f], ref[f], area)
    return out, t


def _log_errors(kind, errs):
    """Appends measured errors to the file named by SWE_ERRLOG (if set), one
    JSON line per comparison with the test that made it."""
    path = os.environ.get("SWE_ERRLOG")
    if not path:
        return
    import json
    with open(path, "a") as f:
        f.write(json.dumps({"test": os.environ.get("PYTEST_CURRENT_TEST", ""), "kind": kind, **errs}) + "\n")


def compare(state, sim, tol, metric="max", max_bound=None):
    """FP64 (metric "max"): every field within tol in the max norm.

    FP32 trajectories (metric "l1"): the area-weighted L1 errors of h, qx
    and qy within tol, and the max errors within max_bound, which is tol
    itself unless a test gives a bound measured on its own workload.  Only
    the 4M-cell comparison does: there, among millions of edges, a few have a
    reconstructed depth H - max(z_L, z_R) within the FP32 rounding of H and z
    (about 1e-6 m) of zero, where the HLLC wave speeds switch from the two-
    rarefaction estimate to the dry-bed form; such an edge takes the other
    branch than the FP64 oracle, its flux differs by O(h c) for a step, and
    the difference spreads and decays over the following steps.  The
    arithmetic of a step itself is held to tol in the max norm there by
    local_step_errors."""
    got = state.read()
    errs, t = errors(got, sim)
    if metric == "max":
        bad = {k: v for k, v in errs.items() if k.startswith("max_") and not v <= tol}
    else:
        if max_bound is None:
            max_bound = tol
        bad = {k: v for k, v in errs.items() if (k.startswith("l1_") and not v <= tol)
               or (k.startswith("max_") and k != "max_H" and not v <= max_bound)}
    _log_errors(metric, errs)
    assert not bad, f"parity beyond {tol} ({metric}, max bound {max_bound}): {errs} (t gpu {got['t']} oracle {t})"
    assert abs(got["t"] - t) <= 1e-9 * max(1.0, abs(t)), (got["t"], t)
    return errs


def oracle_on_fp32_bed(sc, mesh=None, omp=False):
    """The oracle run of scenario sc on the bed an FP32 state carries: each
    cell's bed rounded to single precision, with the initial surface given
    (H0, clamped to that bed) or the initial depth kept (h0).  FP32 and FP64
    arithmetic are then compared on the same input."""
    import oracle
    sim = oracle.Sim(sc, mesh=mesh, omp=omp)
    z32 = sim.bed().astype(np.float32).astype(np.float64)
    if sc.H0 is not None:
        sim.set_bed(z32, np.maximum(np.asarray(sc.H0, np.float64), z32))
    else:
        sim.set_bed(z32)
    return sim


def local_step_errors(state, sc, om=None, steps=1):
    """Max and L1 errors of `steps` GPU steps against the oracle started
    from the GPU's own state on the GPU's own bed (the FP32 values, given to
    the oracle per cell): every wet/dry decision of the first step is then
    taken on identical numbers on both sides, so the difference is the
    arithmetic of the step alone.  The oracle steps with the time step the
    GPU took."""
    import oracle
    got = state.read()
    z = state.bed()
    fixed = S.Scenario(**{**sc.__dict__})
    om = om or oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    sim = oracle.Sim(fixed, mesh=om, t0=got["t"])
    sim.set_bed(z, got["H"])
    sim.set_state(got["H"], got["qx"], got["qy"], got["t"])
    for _ in range(steps):
        dt = state.step()
        sim.step(t_end=sim.t + dt)
    errs, _ = errors(state.read(), sim)
    _log_errors("local", errs)
    return errs
