"""The Exner module on the GPU (section "Morphodynamics": eq. exner, eq.
exnerupdateformula, the HLL sediment flux eq. exner_hll with the speeds of
eq. exner_wave_assign / eq. exner_wave_estimation, Table
sedtransport_closure): parity of the bed and the water with the FP64 oracle
(FP64 within 1e-10 of the norm; FP32 within 1e-4 in the max and L1 norms on a fixed
step) on a closed basin, an open channel with a non-erodible bed, wet/dry
multi-tile meshes with each closure and friction law; sediment conservation;
the lake at rest; the hump's migration at the bed celerity; the API."""
import math

import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import compare, gpu_state, l1_rel, rel_err
from swe_inputs import mesh as M
from test_oracle_morpho import _box, _bumps

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


def _bed_parity(st, sim, tol, metric="max"):
    zg, zo = st.bed(), sim.bed()
    if metric == "max":
        assert rel_err(zg, zo) <= tol, rel_err(zg, zo)
    else:
        assert l1_rel(zg, zo, sim.mesh.geometry()["area"]) <= tol


def _basin():
    return _box(40.0, 10.0, 1.0, lambda x, y: 0.05 * np.sin(x / 3.0), lambda x: np.where(x < 20.0, 1.0, 0.3),
                S.Morpho("mpm", d_m=1e-3))


def test_closed_basin_fp64(swe):
    sc = _basin()
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    v0 = st.morpho_volume()[0]
    z0 = sim.bed()
    for k in range(200):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    compare(st, sim, FP64_TOL)
    _bed_parity(st, sim, FP64_TOL)
    dzg, dzo = st.bed() - z0, sim.bed() - z0
    assert np.abs(dzo).max() > 1e-3 and rel_err(dzg, dzo) <= 1e-6
    v, b, c = st.morpho_volume()
    assert b == 0.0 and c == 0.0 and abs(v - v0) <= 1e-12 * abs(v0) + 1e-13


def test_closed_basin_fp32(swe):
    sc = _basin()
    fixed = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
    st = gpu_state(fixed, swe.FP32)
    sim = oracle.Sim(fixed)
    z0 = sim.bed()
    for _ in range(100):
        st.step()
        sim.step()
    compare(st, sim, FP32_TOL, metric="l1")
    dzg, dzo = st.bed() - z0, sim.bed() - z0
    area = sim.mesh.geometry()["area"]
    assert l1_rel(dzg, dzo, area) <= 1e-2   # the bed change itself, relative to its own size


def _open_channel(prec_fixed=False):
    xy, tri, sides = M.structured_right(60.0, 4.0, 1.0)
    n = len(tri)
    segs = [M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), M.segments_on_side(xy, sides["x1"], -1, 1e9, 1)]
    tags = [np.full(len(segs[0]), 1, np.int32), np.full(len(segs[1]), 2, np.int32)]
    z = 0.002 * (60.0 - xy[:, 0])
    mo = S.Morpho("mpm", z_rel=np.full(n, -2e-4))  # reached by the scour near the inflow
    return S.Scenario("open", np.c_[xy, z], tri.astype(np.int32), np.concatenate(segs), np.concatenate(tags),
                      [S.BC(1, S.INFLOW_UNIFORM, slope=2e-3, t=np.array([0.0]), Q=np.array([6.0])),
                       S.BC(2, S.OUTFLOW_ZEROGRAD)], None, np.full(n, 0.5), np.full(n, 1.0), np.zeros(n),
                      np.full(n, 0.02), t_end=30.0, cfl=0.5, morpho=mo)


def test_open_channel_fixed_bed_fp64(swe):
    sc = _open_channel()
    st = gpu_state(sc, swe.FP64)
    v0 = st.morpho_volume()[0]
    zfix = st.bed() - 2e-4
    st.run_until(30.0)
    sim = oracle.Sim(sc)
    sim.run_until(30.0)
    compare(st, sim, FP64_TOL)
    _bed_parity(st, sim, FP64_TOL)
    v, b, c = st.morpho_volume()
    vo, bo, co = sim.morpho_diag()
    assert abs(b - bo) <= FP64_TOL * abs(bo) and c > 0.0 and abs(c - co) <= 1e-8 * co
    assert np.all(st.bed() >= zfix - 1e-15)
    assert abs(v - (v0 - b + c)) <= 1e-12 * abs(v0)


@pytest.mark.parametrize("closure,friction", [("mpm", "manning"), ("grass", "manning"), ("eh", "chezy"),
                                              ("mpm", "bezzola")])
def test_wet_dry_multi_tile_fp64(swe, closure, friction):
    base = S.tiny_random(25, 13, seed=7)   # 650 cells: two full tiles and a ragged one
    par = {"manning": base.manning, "chezy": np.full(base.n_cells, 0.02),
           "bezzola": np.full(base.n_cells, 0.05)}[friction]
    bcs = base.bcs if friction == "manning" else [S.BC(2, S.OUTFLOW_ZEROGRAD)]
    mo = {"mpm": S.Morpho("mpm", d_m=5e-3), "grass": S.Morpho("grass", alpha=2e-4, m=3.0, thr=0.05),
          "eh": S.Morpho("eh", d_m=0.05)}[closure]
    sc = S.Scenario(**{**base.__dict__, "manning": par, "friction": friction, "bcs": bcs, "morpho": mo})
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    z0 = sim.bed()
    for k in range(20):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    compare(st, sim, FP64_TOL)
    _bed_parity(st, sim, FP64_TOL)
    assert np.abs(sim.bed() - z0).max() > 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lake_at_rest_keeps_the_bed(swe, prec):
    sc = _box(30.0, 10.0, 1.0, _bumps, 1.0, S.Morpho("mpm"))
    st = gpu_state(sc, swe.FP64 if prec == "fp64" else swe.FP32)
    z0 = st.bed()
    for _ in range(100):
        st.step()
    assert np.array_equal(st.bed(), z0)
    r = st.read()
    assert np.all(r["qx"] == 0.0) and np.all(r["qy"] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hump_migrates_at_the_bed_celerity(swe, prec):
    A, p, Fr, h = 5e-3, 0.4, 0.25, 1.0
    G = 9.81
    u = Fr * math.sqrt(G * h)
    xy, tri, sides = M.structured_right(100.0, 2.0, 0.5)
    n = len(tri)
    segs = [M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), M.segments_on_side(xy, sides["x1"], -1, 1e9, 1)]
    tags = [np.full(len(segs[0]), 1, np.int32), np.full(len(segs[1]), 2, np.int32)]
    z = 0.01 * np.exp(-((xy[:, 0] - 30.0) / 4.0) ** 2)
    cx = xy[tri, 0].mean(axis=1)
    mo = S.Morpho("grass", alpha=A, m=3.0, thr=0.0, porosity=p)
    sc = S.Scenario("hump", np.c_[xy, z], tri.astype(np.int32), np.concatenate(segs), np.concatenate(tags),
                    [S.BC(1, S.INFLOW_FROUDE, slope=Fr, t=np.array([0.0]), Q=np.array([2.0 * u * h])),
                     S.BC(2, S.OUTFLOW_ZEROGRAD)], np.full(n, h), None, np.full(n, u * h), np.zeros(n),
                    np.zeros(n), t_end=200.0, cfl=0.5, morpho=mo)
    st = gpu_state(sc, swe.FP64 if prec == "fp64" else swe.FP32)
    area = oracle.Mesh(sc.nodes, sc.tri).geometry()["area"]

    def centre():
        w = np.clip(st.bed(), 0, None) * area
        sel = (cx > 10.0) & (cx < 90.0)
        return (cx[sel] * w[sel]).sum() / w[sel].sum()

    st.run_until(20.0)
    x0, t0 = centre(), st.read()["t"]
    st.run_until(200.0)
    speed = (centre() - x0) / (st.read()["t"] - t0)
    cb = 3.0 * A * u ** 3 / ((1.0 - p) * h * (1.0 - Fr ** 2))
    assert abs(speed - cb) <= 0.05 * cb, (speed, cb)


def test_morpho_api(swe):
    sc = S.tiny_random(4, 3, seed=1)
    st = gpu_state(sc, swe.FP32, block_size=512)
    with pytest.raises(swe.SweError, match="not moving"):
        st.morpho_volume()
    with pytest.raises(swe.SweError, match="bad sediment"):
        st.set_morpho(S.Morpho("mpm", porosity=1.0))
    with pytest.raises(swe.SweError, match="z_rel"):
        st.set_morpho(S.Morpho("mpm", z_rel=np.full(sc.n_cells, 0.1)))
    st.set_morpho(S.Morpho("mpm"))
    assert st.autotune(2) == 256
    with pytest.raises(swe.SweError, match="do not combine"):
        st.set_scalars(np.zeros((1, sc.n_cells)))
    b = swe.Batch(swe.FP32)
    with pytest.raises(swe.SweError, match="not batched"):
        b.add(st, 1.0)
    b.close()
    st.step()
    assert np.all(np.isfinite(st.bed()))
    st.set_morpho(None)
    z = st.bed()
    st.step()
    assert np.array_equal(st.bed(), z)   # the bed no longer moves
