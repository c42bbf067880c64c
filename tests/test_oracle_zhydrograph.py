"""Pins of the prescribed water-surface boundary ("zhydrograph", section
"Hydrodynamic BCs"; reading: the ghost is still water at the prescribed
surface over the boundary cell's bed) in the oracle.

* A lake at rest whose boundary level equals the lake surface stays at rest
  bit for bit (the ghost is the interior state mirrored).
* Water enters or leaves only through the open boundary: the volume change
  equals minus the integrated boundary mass flux to round-off.
* Raising the level fills the basin, lowering it drains it, towards the
  still-water volume of the new level (computed from the bed geometry)."""
import numpy as np

import oracle
import swe_inputs as S


def test_lake_at_boundary_level_stays_at_rest():
    sc = S.level_basin([0.0], [0.625], H0=0.625)
    sim = oracle.Sim(sc)
    H0, _, _, _ = sim.state()
    for _ in range(200):
        sim.step()
    H, qx, qy, _ = sim.state()
    assert np.array_equal(H, H0) and not qx.any() and not qy.any()


def _volume_at(sc, level):
    g = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag).geometry()
    area, zb = g["area"], g["zb"]
    return float(np.sum(np.maximum(level - zb, 0.0) * area)), area, zb


def _run_to(sc, t):
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    sim.run_until(t)
    return sim, m0


def test_fill_and_drain_conserve_and_approach_the_new_level():
    # fill: level rises from 0.3 to 0.9 over 20 s
    sc = S.level_basin([0.0, 20.0], [0.3, 0.9], H0=0.3, t_end=400.0)
    sim, m0 = _run_to(sc, 400.0)
    d = sim.diag()
    assert abs(d["mass"] - (m0 - d["bnd_flux"] + d["clipped"])) <= 1e-11 * d["mass"]
    v_end, area, zb = _volume_at(sc, 0.9)
    assert d["bnd_flux"] < 0 and abs(d["mass"] - v_end) <= 0.02 * v_end, (d, v_end)
    # drain: level drops from 0.9 to 0.4
    sc2 = S.level_basin([0.0, 20.0], [0.9, 0.4], H0=0.9, t_end=400.0)
    sim2, m02 = _run_to(sc2, 400.0)
    d2 = sim2.diag()
    assert abs(d2["mass"] - (m02 - d2["bnd_flux"] + d2["clipped"])) <= 1e-11 * d2["mass"]
    v2, _, _ = _volume_at(sc2, 0.4)
    assert d2["bnd_flux"] > 0 and abs(d2["mass"] - v2) <= 0.02 * v2, (d2, v2)
