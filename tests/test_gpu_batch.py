"""Batched ensembles: many uneven meshes stepped by one persistent kernel per
step, each member with its own time step and end time.  Every member's result
in the batch must equal the same member solved alone, bit for bit (the cell
update is per cell and the time-step minimum is order independent)."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import device, gpu_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


@pytest.fixture(scope="module")
def members():
    sizes = [3000, 12000, 5000, 20000, 1500]
    return [S.ensemble_member(k, n, t_end=60.0) for k, n in enumerate(sizes)]


def _alone(sc, prec, t_end):
    st = gpu_state(sc, prec)
    st.run_until(t_end)
    return st.read()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_alone(swe, members, prec):
    p = swe.FP32 if prec == "fp32" else swe.FP64
    ends = [60.0, 45.0, 60.0, 30.0, 60.0]
    alone = [_alone(sc, p, te) for sc, te in zip(members, ends)]
    batch = swe.Batch(precision=p, device=device())
    states = []
    for sc, te in zip(members, ends):
        st = gpu_state(sc, p)
        states.append(st)
        batch.add(st, te)
    rounds = 0
    while batch.step(16) > 0:
        rounds += 1
        assert rounds < 10000
    for k, (st, ref, te) in enumerate(zip(states, alone, ends)):
        info = batch.poll(k)
        assert info["done"] and info["error"] == 0 and info["t"] == te
        got = st.read()
        for f in ("H", "qx", "qy"):
            assert np.array_equal(got[f], ref[f]), (k, f)
        assert got["t"] == ref["t"]


def test_batch_member_matches_oracle_fp64(swe, members):
    sc = members[0]
    batch = swe.Batch(precision=swe.FP64, device=device())
    st = gpu_state(sc, swe.FP64)
    batch.add(st, 20.0)
    while batch.step(8) > 0:
        pass
    sim = oracle.Sim(sc)
    sim.run_until(20.0)
    got = st.read()
    H, qx, qy, t = sim.state()
    for a, b in ((got["H"], H), (got["qx"], qx), (got["qy"], qy)):
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    assert got["t"] == t


def test_batch_budget_and_remove(swe, members):
    a = gpu_state(members[0], swe.FP32)
    b = gpu_state(members[1], swe.FP32)
    fa = a.mesh.footprint(swe.FP32)
    batch = swe.Batch(precision=swe.FP32, budget_bytes=fa + 1000, device=device())
    slot = batch.add(a, 60.0)
    with pytest.raises(swe.SweError) as e:
        batch.add(b, 60.0)
    assert e.value.code == swe.EBUDGET
    # precision must match
    c = gpu_state(members[2], swe.FP64)
    big = swe.Batch(precision=swe.FP32, device=device())
    with pytest.raises(swe.SweError):
        big.add(c, 10.0)
    # remove mid-run; the state stays usable alone and ends where a solo run ends
    batch.step(5)
    batch.remove(slot)
    assert batch.step(5) == 0
    a.run_until(60.0)
    ref = _alone(members[0], swe.FP32, 60.0)
    got = a.read()
    assert all(np.array_equal(got[f], ref[f]) for f in ("H", "qx", "qy"))


def test_batch_admits_while_running(swe, members):
    # continuous batching: a member added while others are mid-run gives the
    # same result as alone
    p = swe.FP32
    ref = [_alone(members[k], p, 40.0) for k in (0, 2)]
    batch = swe.Batch(precision=p, device=device())
    s0 = gpu_state(members[0], p)
    batch.add(s0, 40.0)
    batch.step(7)
    s2 = gpu_state(members[2], p)
    batch.add(s2, 40.0)
    while batch.step(9) > 0:
        pass
    for st, r in zip((s0, s2), ref):
        got = st.read()
        assert all(np.array_equal(got[f], r[f]) for f in ("H", "qx", "qy"))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_autotune_restores_members(swe, members, prec):
    # the batched autotuner times every tile size on the running members and
    # puts each back exactly as it was: the run continues bitwise like a solo
    # run, whichever tile it picked
    p = swe.FP32 if prec == "fp32" else swe.FP64
    ends = [30.0, 30.0, 20.0]
    alone = [_alone(members[k], p, te) for k, te in zip((0, 1, 4), ends)]
    batch = swe.Batch(precision=p, device=device())
    states = [gpu_state(members[k], p) for k in (0, 1, 4)]
    for st, te in zip(states, ends):
        batch.add(st, te)
    batch.step(5)
    before = [st.read() for st in states]
    tile = batch.autotune(3)
    assert tile in (128, 256, 512)
    for st, b in zip(states, before):
        got = st.read()
        assert all(np.array_equal(got[f], b[f]) for f in ("H", "qx", "qy")) and got["t"] == b["t"]
    while batch.step(8) > 0:
        pass
    for st, ref in zip(states, alone):
        got = st.read()
        assert all(np.array_equal(got[f], ref[f]) for f in ("H", "qx", "qy")) and got["t"] == ref["t"]
        m = st.mass()
        assert m["steps"] > 0
