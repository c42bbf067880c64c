"""Host-side logic of the serving loop (admission by footprint, continuous
batching, latency accounting) against a stub device that only counts bytes
and steps -- no GPU needed."""
import time
import types

import numpy as np
import pytest

from paper_2102_12862_amd import serve


class StubDevice:
    pass


class StubMesh:
    live = 0

    def __init__(self, nodes, tri, seg, tag, device=None):
        self.n_cells = len(tri)
        StubMesh.live += 1

    def footprint(self, precision):
        return 100 * self.n_cells

    def close(self):
        StubMesh.live -= 1


class StubState:
    def __init__(self, mesh, sc, precision=None):
        if getattr(sc, "bad", False):
            raise ValueError("invalid scenario")
        self.n = mesh.n_cells
        self.t = 0.0
        self.steps = 0
        self.dt = sc.dt

    def read(self):
        return {"t": self.t, "n": self.n}

    def close(self):
        pass


class StubBatch:
    def __init__(self, precision=None, budget_bytes=0, device=None):
        self.budget = budget_bytes
        self.members = {}
        self.max_concurrent = 0

    def add(self, st, t_end):
        slot = 0
        while slot in self.members:
            slot += 1
        self.members[slot] = (st, t_end)
        self.max_concurrent = max(self.max_concurrent, len(self.members))
        return slot

    def remove(self, slot):
        del self.members[slot]

    def step(self, k):
        time.sleep(0.0005)  # a round of device work takes time
        for st, te in self.members.values():
            for _ in range(k):
                if st.t < te:
                    st.t = min(te, st.t + st.dt)
                    st.steps += 1
        return sum(st.t < te for st, te in self.members.values())

    def poll(self, slot):
        st, te = self.members[slot]
        return {"done": st.t >= te, "error": 0, "t": st.t, "steps": st.steps}

    def close(self):
        pass


@pytest.fixture
def stubbed(monkeypatch):
    fake = types.SimpleNamespace(Mesh=StubMesh, State=StubState, Batch=StubBatch, TorchDevice=StubDevice,
                                 FP32=1, FP64=0)
    monkeypatch.setattr(serve, "swe", fake)
    return fake


def make(n, dt=1.0):
    sc = types.SimpleNamespace(nodes=np.zeros((3, 3)), tri=np.zeros((n, 3)), bnd_seg=None, bnd_tag=None,
                               dt=dt, n_cells=n)
    return lambda: sc


def test_all_requests_complete_and_budget_binds(stubbed):
    reqs = [serve.Request(i, arrival=0.001 * i, make=make(1000 * (i + 1)), t_end=10.0 * (i + 1))
            for i in range(6)]
    srv = serve.Server(budget_bytes=100 * 7000, steps_per_round=4, device=StubDevice())
    srv.serve(reqs)
    for r in reqs:
        assert r.error is None and r.finished is not None and r.result["t"] == r.t_end
        assert r.admitted >= r.arrival and r.finished >= r.admitted
        assert r.steps == int(r.t_end)
    # never more resident than the budget allows
    assert srv.batch.max_concurrent <= 3
    s = serve.summarize(reqs, wall=max(r.finished for r in reqs))
    assert s["requests"] == 6 and s["errors"] == 0 and s["p99_s"] >= s["p50_s"] > 0


def test_oversized_request_is_refused_not_hung(stubbed):
    reqs = [serve.Request(0, 0.0, make(10), 3.0), serve.Request(1, 0.0, make(10 ** 6), 3.0),
            serve.Request(2, 0.0, make(20), 3.0)]
    srv = serve.Server(budget_bytes=100 * 1000, steps_per_round=2, device=StubDevice())
    srv.serve(reqs)
    assert reqs[0].error is None and reqs[2].error is None
    assert "budget" in reqs[1].error


def test_late_arrivals_join_running_batch(stubbed):
    reqs = [serve.Request(0, 0.0, make(100, dt=0.001), 5.0), serve.Request(1, 0.02, make(100, dt=0.001), 1.0)]
    srv = serve.Server(budget_bytes=0, steps_per_round=50, device=StubDevice())
    srv.serve(reqs)
    assert reqs[1].admitted < reqs[0].finished  # joined while request 0 was running
    assert srv.batch.max_concurrent == 2


def test_failing_request_is_reported_and_freed(stubbed):
    bad = make(50)
    bad().bad = True
    reqs = [serve.Request(0, 0.0, make(10), 3.0), serve.Request(1, 0.0, bad, 3.0),
            serve.Request(2, 0.0, make(10 ** 6), 3.0), serve.Request(3, 0.001, make(20), 3.0)]
    StubMesh.live = 0
    srv = serve.Server(budget_bytes=100 * 1000, steps_per_round=2, device=StubDevice())
    srv.serve(reqs)
    assert reqs[0].error is None and reqs[3].error is None
    assert "invalid scenario" in reqs[1].error and "budget" in reqs[2].error
    assert all(r.finished is not None for r in reqs)
    assert StubMesh.live == 0  # every mesh, admitted or refused, was closed
