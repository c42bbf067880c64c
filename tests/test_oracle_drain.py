"""Pins of the draining-time positivity limiter in the oracle (an option that
replaces the positivity clip of the update: every flux leaving a cell
acts only for that cell's draining time h |Omega| / (its outgoing mass flux)):

* no cell drains in a wet flow, so the limiter changes nothing (bitwise);
* a lake at rest is untouched (bitwise);
* where the bare scheme clips (wet/dry flows, a wet cell on a dry bed), the
  limiter leaves depths >= 0 with a clip of rounding size and conserves the
  volume: M(t) = M(0) - outflow to round-off;
* a single wet column on a dry bed keeps exactly its volume (the bare clip
  adds most of it again);
* the Ritter dam break keeps its front: the limited and bare solutions agree
  to a few percent in L1 away from the tip.
"""
import numpy as np

import oracle
import swe_inputs as S
from swe_inputs import mesh as M


def _with(sc, **kw):
    return S.Scenario(**{**sc.__dict__, **kw})


def test_wet_flow_is_unchanged():
    sc = S.dam_break(d=1.0, h_right=0.1)
    a, b = oracle.Sim(sc), oracle.Sim(_with(sc, drain=True))
    for _ in range(60):
        assert a.step() == b.step()
    for x, y in zip(a.state()[:3], b.state()[:3]):
        assert np.array_equal(x, y)


def test_lake_at_rest_is_untouched():
    sc = S.lake_at_rest(n_cells=3000)
    sim = oracle.Sim(_with(sc, drain=True))
    H0 = sim.state()[0]
    for _ in range(50):
        sim.step()
    H, qx, qy, _ = sim.state()
    assert np.array_equal(H, H0) and np.all(qx == 0.0) and np.all(qy == 0.0)


def test_wet_dry_flows_keep_positive_depths_without_clipping():
    clipped_bare = 0.0
    for seed in (0, 2, 4, 5):
        sc = S.tiny_random(6, 4, seed=seed)
        bare = oracle.Sim(sc)
        sim = oracle.Sim(_with(sc, drain=True))
        m0 = sim.diag()["mass"]
        for _ in range(30):
            bare.step()
            sim.step()
            h = sim.state()[0] - sim.bed()
            assert h.min() >= 0.0
        clipped_bare += bare.diag()["clipped"]
        d = sim.diag()
        assert d["clipped"] <= 1e-15 * m0, d["clipped"]
        assert abs(d["mass"] - (m0 - d["bnd_flux"])) <= 1e-13 * m0
    assert clipped_bare > 0.05   # the bare scheme does clip on these flows


def test_single_column_on_a_dry_bed_keeps_its_volume():
    xy, tri, _ = M.structured_right(10.0, 10.0, 1.0)
    n = len(tri)
    cx, cy = xy[tri, 0].mean(axis=1), xy[tri, 1].mean(axis=1)
    h0 = np.where((np.abs(cx - 5.3) < 0.4) & (np.abs(cy - 5.6) < 0.4), 1.0, 0.0)
    sc = S.Scenario("column", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                    np.zeros(0, np.int32), [], None, h0, np.zeros(n), np.zeros(n), np.zeros(n), t_end=1.0, cfl=0.9)
    bare, sim = oracle.Sim(sc), oracle.Sim(_with(sc, drain=True))
    v0 = sim.diag()["mass"]
    for _ in range(5):
        bare.step()
        sim.step()
    assert bare.diag()["clipped"] > 0.5 * v0          # the clip makes up most of the volume again
    d = sim.diag()
    assert d["clipped"] == 0.0 and abs(d["mass"] - v0) <= 1e-15 * v0
    assert (sim.state()[0] - sim.bed()).min() >= 0.0


def test_ritter_front_is_kept():
    sc = S.dam_break(d=0.5, h_right=0.0, t_end=4.0)
    bare, sim = oracle.Sim(sc), oracle.Sim(_with(sc, drain=True))
    bare.run_until(4.0)
    sim.run_until(4.0)
    area = sim.mesh.geometry()["area"]
    hb = bare.state()[0] - bare.bed()
    hd = sim.state()[0] - sim.bed()
    cx = sc.centroids()[:, 0]
    body = cx < 75.0      # the rarefaction and the thin front region up to the tip's neighbourhood
    assert (np.abs(hd - hb) * area)[body].sum() <= 0.02 * (hb * area)[body].sum()
    assert sim.diag()["clipped"] <= 1e-15 * sim.diag()["mass"]
