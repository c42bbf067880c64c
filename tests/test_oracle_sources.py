"""Pins of the external water sources and sinks S_h in the oracle (the S_h
paragraph of the hydrodynamic closure relations; eq.
swe_vectorial_form_sourceterms, an explicit source in the continuity equation
of eq. hydrodynamicupdateformula):

* uniform rain (intensity in mm/h) on a closed flat basin raises a lake at
  rest by exactly the rain depth, and keeps it at rest;
* a total discharge spread over a region adds Q dt per step, with the
  series taken at t^n (checked against the recorded step sequence);
* an exact sink drains linearly, and one larger than the water is an error;
* an available sink empties cells to exactly dry without a clip;
* an infinity sink keeps its region dry while water flows in;
* sinks keep the concentration of passive species, sources dilute it;
* the volume balance M(t) = M(0) - outflow + clipped + source volume holds
  to round-off on a wet/dry flow with all three modes.
"""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M


def _basin(h0=0.5, lx=20.0, ly=10.0, d=1.0, **kw):
    xy, tri, _ = M.structured_right(lx, ly, d)
    n = len(tri)
    base = dict(name="basin", nodes=np.c_[xy, np.zeros(len(xy))], tri=tri.astype(np.int32),
                bnd_seg=np.zeros((0, 2), np.int32), bnd_tag=np.zeros(0, np.int32), bcs=[], H0=None,
                h0=np.full(n, h0), qx0=np.zeros(n), qy0=np.zeros(n), manning=np.full(n, 0.02), t_end=100.0,
                dt_max=0.5, cfl=0.5)
    base.update(kw)
    return S.Scenario(**base)


def _everywhere(sc, src):
    return S.Scenario(**{**sc.__dict__, "sources": (src,), "src_region": np.zeros(sc.n_cells, np.int32)})


def _state(sim):
    H, qx, qy, t = sim.state()
    zb = sim.mesh.geometry()["zb"]
    return H - zb, qx, qy, t


def test_uniform_rain_raises_a_lake_at_rest():
    sc = _everywhere(_basin(), S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([36.0])))
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    sim.run_until(50.0)
    h, qx, qy, t = _state(sim)
    assert t == 50.0
    assert np.all(qx == 0.0) and np.all(qy == 0.0)          # still at rest
    assert np.ptp(h) == 0.0                                   # level everywhere
    assert abs(h[0] - (0.5 + 1e-5 * 50.0)) <= 1e-13            # 36 mm/h = 1e-5 m/s
    area = 20.0 * 10.0
    assert abs(sim.source_volume() - 1e-5 * 50.0 * area) <= 1e-12 * area
    d = sim.diag()
    assert abs(d["mass"] - m0 - sim.source_volume()) <= 1e-12 * m0


def test_discharge_over_a_region_follows_the_series_at_t_n():
    sc = _basin(h0=0.3)
    cx = sc.centroids()[:, 0]
    region = np.where(cx < 5.0, 0, -1).astype(np.int32)
    # Q(t) = 1 + 0.2 t (linear between the two points, constant after t = 30)
    src = S.Source(S.SRC_EXACT, S.SRC_DISCHARGE, np.array([0.0, 30.0]), np.array([1.0, 7.0]))
    sim = oracle.Sim(S.Scenario(**{**sc.__dict__, "sources": (src,), "src_region": region}))
    expect = 0.0
    while sim.t < 40.0:
        t = sim.t
        dt = sim.step()
        expect += min(1.0 + 0.2 * t, 7.0) * dt
    assert abs(sim.source_volume() - expect) <= 1e-12 * expect
    d = sim.diag()
    m0 = 0.3 * 200.0
    assert abs(d["mass"] - (m0 + expect)) <= 1e-12 * m0
    # the water went into the region first
    h = _state(sim)[0]
    assert h[cx < 5.0].mean() > h[cx > 15.0].mean()


def test_exact_sink_drains_linearly():
    sc = _everywhere(_basin(), S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([-36.0])))
    sim = oracle.Sim(sc)
    sim.run_until(40.0)
    h = _state(sim)[0]
    assert np.ptp(h) == 0.0 and abs(h[0] - (0.5 - 1e-5 * 40.0)) <= 1e-13


def test_exact_sink_beyond_the_water_is_an_error():
    sc = _everywhere(_basin(h0=0.01), S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([-3.6e6])))
    sim = oracle.Sim(sc)
    with pytest.raises(oracle.OracleError) as e:
        sim.step()   # dt 0.5 s at 1 m/s removes 0.5 m of 0.01 m
    assert e.value.code == -8
    h = _state(sim)[0]
    assert np.all(h == 0.0)
    assert sim.diag()["clipped"] > 0.0


def test_available_sink_empties_to_exactly_dry():
    sc = _everywhere(_basin(h0=0.01), S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]),
                                               np.array([-3.6e6])))
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    sim.step()
    H, _, _, _ = sim.state()
    zb = sim.mesh.geometry()["zb"]
    assert np.array_equal(H, zb)
    d = sim.diag()
    assert d["clipped"] == 0.0 and d["mass"] == 0.0
    assert abs(sim.source_volume() + m0) <= 1e-15 * m0


def test_available_sink_only_removes():
    sc = _everywhere(_basin(), S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]), np.array([5.0])))
    with pytest.raises(oracle.OracleError, match="only exact"):
        oracle.Sim(sc)


def test_empty_discharge_region_is_rejected():
    sc = _basin()
    src = S.Source(S.SRC_EXACT, S.SRC_DISCHARGE, np.array([0.0]), np.array([1.0]))
    with pytest.raises(oracle.OracleError, match="empty"):
        oracle.Sim(S.Scenario(**{**sc.__dict__, "sources": (src,),
                                 "src_region": np.full(sc.n_cells, -1, np.int32)}))


def test_infinity_sink_keeps_its_region_dry():
    base = S.dam_break(d=1.0, h_right=0.0)
    cx = base.centroids()[:, 0]
    region = np.where(cx > 80.0, 0, -1).astype(np.int32)
    sc = S.Scenario(**{**base.__dict__, "sources": (S.Source(S.SRC_INFINITY),), "src_region": region})
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    steps = 0
    while sim.t < 8.0:
        sim.step()
        steps += 1
        h = _state(sim)[0]
        assert np.all(h[cx > 80.0] == 0.0)
    assert sim.source_volume() < 0.0    # the front reached the sink
    d = sim.diag()
    assert abs(d["mass"] - (m0 - d["bnd_flux"] + d["clipped"] + sim.source_volume())) <= 1e-12 * m0


def test_species_follow_sinks_and_sources():
    n = _basin().n_cells
    rain = _everywhere(_basin(), S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([3600.0])))
    sim = oracle.Sim(S.Scenario(**{**rain.__dict__, "phi0": np.full((1, n), 0.3)}))
    sim.run_until(20.0)
    h = _state(sim)[0]
    phi = sim.scalars()[0] / h
    assert abs(h[0] - 0.52) <= 1e-13                  # 1 mm/s for 20 s
    assert np.max(np.abs(phi - 0.3 * 0.5 / 0.52)) <= 1e-13   # diluted
    drain = _everywhere(_basin(), S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]), np.array([-3600.0])))
    sim = oracle.Sim(S.Scenario(**{**drain.__dict__, "phi0": np.full((1, n), 0.3)}))
    sim.run_until(20.0)
    h = _state(sim)[0]
    assert abs(h[0] - 0.48) <= 1e-13
    assert np.max(np.abs(sim.scalars()[0] / h - 0.3)) <= 1e-13   # kept


def test_balance_with_all_modes_on_a_wet_dry_flow():
    sc = S.tiny_random(6, 4, seed=3)
    n = sc.n_cells
    r = np.random.default_rng(9)
    region = r.integers(-1, 3, n).astype(np.int32)
    srcs = (S.Source(S.SRC_EXACT, S.SRC_DISCHARGE, np.array([0.0, 0.5]), np.array([0.4, -0.05])),
            S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]), np.array([-2.0e4])),
            S.Source(S.SRC_INFINITY))
    sim = oracle.Sim(S.Scenario(**{**sc.__dict__, "sources": srcs, "src_region": region,
                                   "phi0": r.uniform(0, 1, (2, n))}))
    m0 = sim.diag()["mass"]
    sm0 = sim.scalar_diag()[0]
    for _ in range(25):
        try:
            sim.step()
        except oracle.OracleError as e:
            assert e.code == -8   # the exact sink may overdraw a thin cell
    d = sim.diag()
    assert sim.source_volume() != 0.0
    assert abs(d["mass"] - (m0 - d["bnd_flux"] + d["clipped"] + sim.source_volume())) <= 1e-12 * m0
    h = _state(sim)[0]
    assert np.all(h[region == 2] <= 0.0)
    q = sim.scalars()
    assert np.all(q[:, h <= 0.0] == 0.0) and np.all(q >= -1e-15) and np.all(sm0 > 0)
