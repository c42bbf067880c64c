"""Continuous-batching solve service on one GPU.

Flood-scenario solve requests arrive over time (the paper motivates ensemble,
calibration and batch runs of the hydrodynamic model).  The server admits a
request as soon as its HBM footprint fits the budget, keeps its state resident
on the device, and advances every admitted request together: one persistent
kernel per step (``swe_batch_*``), each request with its own time step and end
time.  Requests that arrive while others are on the GPU join at the next
round; finished ones are read back, their memory is released and their
latency (arrival to result on the host) recorded.

Host-side mesh preparation (``swe_mesh_create``, no device work) runs in a
worker thread so it overlaps device work; everything else is issued from the
serving thread on the device's stream.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import swe


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the trace
    make: Callable[[], object]     # returns a scenario (swe_inputs.Scenario)
    t_end: float
    mesh: Optional[swe.Mesh] = None  # a prepared mesh from a cached pool (shared, not closed here)
    admitted: Optional[float] = None
    finished: Optional[float] = None
    cells: int = 0
    steps: int = 0
    result: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class Server:
    def __init__(self, precision=swe.FP32, budget_bytes: int = 2 << 30, steps_per_round: int = 32,
                 device: Optional[swe.TorchDevice] = None, keep_results: bool = True, prep_workers: int = 2):
        self.device = device or swe.TorchDevice()
        self.precision = precision
        self.budget = budget_bytes
        self.k = steps_per_round
        self.keep = keep_results
        self.batch = swe.Batch(precision=precision, budget_bytes=budget_bytes, device=self.device)
        self.pool = cf.ThreadPoolExecutor(max_workers=prep_workers)
        self.rounds = 0
        self.cell_steps = 0

    def _prepare(self, req: Request):
        sc = req.make()
        if req.mesh is not None:
            return sc, req.mesh
        mesh = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=self.device)
        return sc, mesh

    @staticmethod
    def _release(req: Request, mesh):
        if mesh is not None and mesh is not req.mesh:
            mesh.close()

    def serve(self, requests: List[Request], clock=time.perf_counter, idle_sleep: float = 0.0005):
        """Runs the trace in real time and returns the requests with their
        timings filled in."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        prepared: Dict[int, cf.Future] = {}
        waiting: collections.deque = collections.deque()   # arrived, prepared or preparing
        active: Dict[int, tuple] = {}                       # slot -> (req, state, mesh)
        used = 0
        t0 = clock()
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                prepared[r.rid] = self.pool.submit(self._prepare, r)
                waiting.append(r)
            # admission in arrival order, by footprint
            while waiting and prepared[waiting[0].rid].done():
                r = waiting[0]

                def drop(msg, mesh=None, st=None):
                    # an invalid or oversized request is reported and dropped; its
                    # device objects are freed
                    r.error = msg
                    r.finished = clock() - t0
                    if st is not None:
                        st.close()
                    self._release(r, mesh)
                    waiting.popleft()
                    del prepared[r.rid]

                try:
                    sc, mesh = prepared[r.rid].result()
                except Exception as e:
                    drop(str(e))
                    continue
                need = mesh.footprint(self.precision)
                if self.budget and used + need > self.budget:
                    if not active:
                        drop(f"footprint {need} exceeds the budget {self.budget}", mesh)
                        continue
                    break
                st = None
                try:
                    st = swe.State(mesh, sc, precision=self.precision)
                    slot = self.batch.add(st, r.t_end)
                except Exception as e:
                    drop(str(e), mesh, st)
                    continue
                used += need
                r.admitted = clock() - t0
                r.cells = sc.n_cells
                active[slot] = (r, st, mesh, need)
                waiting.popleft()
                del prepared[r.rid]
            if not active:
                if pending:
                    wait = pending[0].arrival - (clock() - t0)
                    if wait > 0 and not waiting:
                        time.sleep(min(wait, 0.01))
                else:
                    time.sleep(idle_sleep)
                continue
            self.batch.step(self.k)
            self.rounds += 1
            for slot in list(active):
                info = self.batch.poll(slot)
                if not info["done"]:
                    continue
                r, st, mesh, need = active.pop(slot)
                r.steps = info["steps"]
                self.cell_steps += r.steps * r.cells
                if info["error"]:
                    r.error = f"solver error {info['error']}"
                elif self.keep:
                    r.result = st.read()
                else:
                    st.read()  # the result still comes back to the host
                r.finished = clock() - t0
                self.batch.remove(slot)
                st.close()
                self._release(r, mesh)
                used -= need
        return requests

    def close(self):
        self.pool.shutdown(wait=True)
        self.batch.close()


def serve_sequential(requests: List[Request], precision=swe.FP32, device=None, clock=time.perf_counter):
    """The same trace served one request at a time (each solved alone with
    swe_run_until, in arrival order) -- the baseline for the served numbers."""
    device = device or swe.TorchDevice()
    t0 = clock()
    for r in sorted(requests, key=lambda r: r.arrival):
        now = clock() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        sc = r.make()
        mesh = r.mesh or swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=device)
        st = swe.State(mesh, sc, precision=precision)
        r.admitted = clock() - t0
        r.steps = st.run_until(r.t_end)
        r.cells = sc.n_cells
        r.result = st.read()
        r.finished = clock() - t0
        st.close()
        if mesh is not r.mesh:
            mesh.close()
    return requests


def summarize(requests: List[Request], wall: float):
    lat = np.array([r.latency for r in requests if r.latency is not None and r.error is None])
    cells = sum(r.cells * r.steps for r in requests if r.error is None)
    return {
        "requests": len(requests),
        "errors": sum(r.error is not None for r in requests),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_s": float(lat.mean()) if len(lat) else None,
        "requests_per_s": len(lat) / wall if wall > 0 else None,
        "cell_updates_per_s": cells / wall if wall > 0 else None,
        "wall_s": wall,
    }
