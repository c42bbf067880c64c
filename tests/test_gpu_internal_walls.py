"""Internal static and dynamic walls and rating curves on the GPU (section
"Hydrodynamic BCs", internal BCs on tagged interior edges): parity with the
FP64 oracle (FP64 within 1e-10 of the norm, FP32 within 1e-4 in the max and
L1 norms on a fixed step) at every tile size, through a dynamic wall's
collapse (at its time, or at the end of the first step that starts with a
cell next to it at its collapse depth, inside the domain and on its
boundary), with species, the Exner module, the draining-time limiter and in a
batch; a rating curve draining one half of a basin into the other, either
way round, with species and in a batch, the volume exact on the device; the
tile edge lists stay consistent; other kinds on interior edges, and a
rating curve with the limiter, are refused."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import compare, device, gpu_state, rel_err
from test_oracle_internal_walls import _cut_basin, _rating_basin, _scenario

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


def _basin(bc, xcut=20.0, lx=40.0, **kw):
    xy, tri, seg = _cut_basin(lx=lx, xcut=xcut)
    cx = xy[tri, 0].mean(axis=1)
    H0 = np.where(cx < 10.0, 1.0, 0.4)
    z = 0.05 * np.sin(xy[:, 0] / 3.0)
    sc = _scenario(xy, tri, seg, np.full(len(seg), 9, np.int32), [bc], H0, z)
    return S.Scenario(**{**sc.__dict__, **kw})


@pytest.mark.parametrize("tile", [128, 256, 512])
def test_static_wall_fp64(swe, tile):
    sc = _basin(S.BC(9, S.WALL))
    st = gpu_state(sc, swe.FP64, block_size=tile)
    st.mesh.check(tile)
    sim = oracle.Sim(sc)
    for k in range(60):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    compare(st, sim, FP64_TOL)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dynamic_wall_collapse(swe, prec):
    sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=2.0), xcut=20.0)
    if prec == "fp64":
        st = gpu_state(sc, swe.FP64)
        st.run_until(6.0)
        sim = oracle.Sim(sc)
        sim.run_until(6.0)
        compare(st, sim, FP64_TOL)
    else:
        fixed = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
        st = gpu_state(fixed, swe.FP32)
        sim = oracle.Sim(fixed)
        while sim.t < 4.0:
            st.step()
            sim.step()
        compare(st, sim, FP32_TOL, metric="l1")


def test_with_species_morpho_and_limiter_fp64(swe):
    n = len(_cut_basin()[1])
    r = np.random.default_rng(5)
    for kw in ({"phi0": r.uniform(0, 1, (2, n))}, {"morpho": S.Morpho("mpm", d_m=1e-3)}, {"drain": True}):
        sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=1.0), **kw)
        st = gpu_state(sc, swe.FP64)
        sim = oracle.Sim(sc)
        for _ in range(40):
            st.step()
            sim.step()
        compare(st, sim, FP64_TOL)
        if "phi0" in kw:
            q, qo = st.scalars(), sim.scalars()
            assert all(rel_err(q[c], qo[c]) <= FP64_TOL for c in range(2))
        if "morpho" in kw:
            assert rel_err(st.bed(), sim.bed()) <= FP64_TOL


def test_batch_matches_a_single_run(swe):
    sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=1.0))
    one = gpu_state(sc, swe.FP32, block_size=256)
    mine = gpu_state(sc, swe.FP32, block_size=256)
    b = swe.Batch(swe.FP32, device=device())
    b.add(mine, 3.0)
    while b.step(16):
        pass
    one.run_until(3.0)
    ra, rb = one.read(), mine.read()
    assert ra["t"] == rb["t"]
    for f in ("H", "qx", "qy"):
        assert np.array_equal(ra[f], rb[f]), f
    b.close()


@pytest.mark.parametrize("tile", [128, 512])
def test_dynamic_wall_collapse_depth_fp64(swe, tile):
    # the dam-break wave raises the cut's cells from 0.4 m to 0.6 m at t ~ 3 s
    sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=1e30, par=0.6))
    st = gpu_state(sc, swe.FP64, block_size=tile)
    sim = oracle.Sim(sc)
    for k in range(150):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    assert sim.t > 6.0
    compare(st, sim, FP64_TOL)
    # water crossed the cut
    wall = oracle.Sim(_basin(S.BC(9, S.WALL)))
    wall.run_until(sim.t)
    assert rel_err(sim.state()[0], wall.state()[0]) > 1e-3


def test_dynamic_wall_collapse_depth_on_the_boundary_fp64(swe):
    base = S.dam_break(d=1.0, h_right=0.0)
    xy = base.nodes[:, :2]
    right = np.where(np.abs(xy[:, 0] - 100.0) < 1e-9)[0]
    right = right[np.argsort(xy[right, 1])]
    seg = np.c_[right[:-1], right[1:]].astype(np.int32)
    sc = S.Scenario(**{**base.__dict__, "bnd_seg": seg, "bnd_tag": np.full(len(seg), 7, np.int32),
                       "bcs": [S.BC(7, S.DYNAMIC_WALL, slope=1e30, par=0.05)]})
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    while sim.t < 20.0:
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (sim.t, dg, do)
    compare(st, sim, FP64_TOL)
    bg, bo = st.mass()["bnd_flux"], sim.diag()["bnd_flux"]
    assert bo > 0.0 and abs(bg - bo) <= 1e-10 * bo, (bg, bo)


def test_dynamic_wall_collapse_depth_fp32_and_batch(swe):
    sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=1e30, par=0.6))
    fixed = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
    st = gpu_state(fixed, swe.FP32)
    sim = oracle.Sim(fixed)
    while sim.t < 6.0:
        st.step()
        sim.step()
    compare(st, sim, FP32_TOL, metric="l1")
    one = gpu_state(sc, swe.FP32, block_size=256)
    mine = gpu_state(sc, swe.FP32, block_size=256)
    b = swe.Batch(swe.FP32, device=device())
    b.add(mine, 8.0)
    while b.step(16):
        pass
    one.run_until(8.0)
    ra, rb = one.read(), mine.read()
    assert ra["t"] == rb["t"]
    for f in ("H", "qx", "qy"):
        assert np.array_equal(ra[f], rb[f]), f
    b.close()


def test_dynamic_wall_collapse_depth_api(swe):
    sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=1.0, par=-0.1))
    m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    with pytest.raises(swe.SweError, match="collapse depth"):
        swe.State(m, sc, precision=swe.FP64)


def test_dynamic_wall_collapse_depth_survives_autotune(swe):
    # the autotuners' trial steps, from t = 1 s, reach the collapse depth at
    # the cut at t = 3.27 s; the runs, with a sink set after the trials,
    # reach it only at t = 3.50 s: the wall's record must come back from
    # the trials as it was
    sc = _basin(S.BC(9, S.DYNAMIC_WALL, slope=1e30, par=0.6))
    region = np.where(sc.centroids()[:, 0] < 20.0, 0, -1)
    sink = [S.Source(S.SRC_AVAILABLE, S.SRC_DISCHARGE, t=np.array([0.0, 1e9]), v=np.array([-10.0, -10.0]))]
    st = gpu_state(sc, swe.FP64, block_size=256)
    other = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    for x in (st, other, sim):
        x.run_until(1.0)
    st.autotune(64)
    b = swe.Batch(swe.FP64, device=device())
    b.add(other, 1e9)
    b.autotune(64)
    b.close()
    for x in (st, other, sim):
        x.set_sources(region, sink)
    for k in range(80):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
        other.step()
    assert sim.t > 4.0
    compare(st, sim, FP64_TOL)
    compare(other, sim, FP64_TOL)


def test_only_walls_on_interior_edges(swe):
    sc = _basin(S.BC(9, S.OUTFLOW_ZEROGRAD))
    m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    with pytest.raises(swe.SweError, match="interior edges"):
        swe.State(m, sc, precision=swe.FP32)


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("tile", [128, 512])
def test_rating_curve_fp64(swe, reverse, tile):
    sc, up = _rating_basin(reverse)
    st = gpu_state(sc, swe.FP64, block_size=tile)
    st.mesh.check(tile)
    v0 = st.mass()["mass"]
    sim = oracle.Sim(sc)
    for k in range(150):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    compare(st, sim, FP64_TOL)
    m = st.mass()
    assert m["bnd_flux"] == 0.0 and abs(m["mass"] - v0) <= 1e-12 * v0
    # water went downstream
    h = st.read()["h"]
    area = sim.mesh.geometry()["area"]
    assert (h * area)[~up].sum() > 0.5 * area[~up].sum() + 1.0


def test_rating_curve_with_species_fp64(swe):
    sc, up = _rating_basin(phi=True)
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    for _ in range(100):
        st.step()
        sim.step()
    compare(st, sim, FP64_TOL)
    q, qo = st.scalars(), sim.scalars()
    assert rel_err(q[0], qo[0]) <= FP64_TOL
    m, b, c = st.scalar_mass()
    mo, bo, co = sim.scalar_diag()
    assert abs(m[0] - mo[0]) <= 1e-12 * mo[0] and b[0] == 0.0


def test_rating_curve_fp32_and_batch(swe):
    sc, up = _rating_basin()
    fixed = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
    st = gpu_state(fixed, swe.FP32)
    sim = oracle.Sim(fixed)
    for _ in range(100):
        st.step()
        sim.step()
    compare(st, sim, FP32_TOL, metric="l1")
    # in a batch, bitwise the single run
    one = gpu_state(sc, swe.FP32, block_size=256)
    mine = gpu_state(sc, swe.FP32, block_size=256)
    b = swe.Batch(swe.FP32, device=device())
    b.add(mine, 20.0)
    while b.step(16):
        pass
    one.run_until(20.0)
    ra, rb = one.read(), mine.read()
    for f in ("H", "qx", "qy"):
        assert np.array_equal(ra[f], rb[f]), f
    b.close()


def test_rating_curve_refuses_the_limiter(swe):
    sc, _ = _rating_basin()
    sc.drain = True
    m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    with pytest.raises(swe.SweError, match="do not combine"):
        swe.State(m, sc, precision=swe.FP64)
