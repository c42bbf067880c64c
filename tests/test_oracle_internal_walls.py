"""Pins of the internal conditions in the oracle (section "Hydrodynamic
BCs": internal static walls and dynamic walls on tagged interior edges):

* a basin cut by a static internal wall evolves, on each side, bitwise like
  that side meshed alone with walls on its cut;
* a dynamic wall stands until its collapse time, then the flow is bitwise
  the flow without the wall restarted from the state at that time;
* only walls and dynamic walls are taken on interior edges.
"""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M


def _cut_basin(lx=40.0, ly=10.0, d=1.0, xcut=20.0):
    """Structured basin with the interior edges on x = xcut tagged 9."""
    xy, tri, _ = M.structured_right(lx, ly, d)
    col = np.where(np.abs(xy[:, 0] - xcut) < 1e-9)[0]
    col = col[np.argsort(xy[col, 1])]
    seg = np.c_[col[:-1], col[1:]].astype(np.int32)
    return xy, tri, seg


def _scenario(xy, tri, seg, tags, bcs, H0, z=None):
    n = len(tri)
    zz = np.zeros(len(xy)) if z is None else z
    return S.Scenario("cut", np.c_[xy, zz], tri.astype(np.int32), seg, tags, bcs, H0, None, np.zeros(n),
                      np.zeros(n), np.full(n, 0.02), t_end=10.0, cfl=0.5)


def test_static_wall_splits_the_basin_bitwise():
    xy, tri, seg = _cut_basin()
    cx = xy[tri, 0].mean(axis=1)
    H0 = np.where(cx < 10.0, 1.0, 0.4)
    z = 0.05 * np.sin(xy[:, 0] / 3.0)
    # the left half alone: its cells in the same order, walls everywhere
    left = cx < 20.0
    keep_nodes = np.unique(tri[left])
    remap = -np.ones(len(xy), np.int64)
    remap[keep_nodes] = np.arange(len(keep_nodes))
    tri_l = remap[tri[left]].astype(np.int32)
    # both on one fixed step (the CFL step is a global minimum)
    sc_full = _scenario(xy, tri, seg, np.full(len(seg), 9, np.int32), [S.BC(9, S.WALL)], H0, z)
    sc_half = _scenario(xy[keep_nodes], tri_l, np.zeros((0, 2), np.int32), np.zeros(0, np.int32), [], H0[left],
                        z[keep_nodes])
    dtf = 0.5 * min(oracle.Sim(sc_full).next_dt(), oracle.Sim(sc_half).next_dt())
    a = oracle.Sim(S.Scenario(**{**sc_full.__dict__, "dt_max": dtf}))
    b = oracle.Sim(S.Scenario(**{**sc_half.__dict__, "dt_max": dtf}))
    for _ in range(80):
        a.step()
        b.step()
    for x, y in zip(a.state()[:3], b.state()[:3]):
        assert np.array_equal(x[left], y)
    # the right side never saw the left side's water
    assert np.all(a.state()[0][~left] <= 0.4 + 0.06)


def test_dynamic_wall_collapses_into_a_plain_edge():
    xy, tri, seg = _cut_basin()
    cx = xy[tri, 0].mean(axis=1)
    H0 = np.where(cx < 20.0, 1.0, 0.3)
    tags = np.full(len(seg), 9, np.int32)
    dyn = oracle.Sim(_scenario(xy, tri, seg, tags, [S.BC(9, S.DYNAMIC_WALL, slope=2.0)], H0))
    static = oracle.Sim(_scenario(xy, tri, seg, tags, [S.BC(9, S.WALL)], H0))
    while dyn.t < 2.0:
        assert dyn.step() == static.step()
    for x, y in zip(dyn.state()[:3], static.state()[:3]):
        assert np.array_equal(x, y)
    # from the collapse on: the flow without the wall, restarted from this state
    H, qx, qy, t = dyn.state()
    free = oracle.Sim(_scenario(xy, tri, seg, tags, [], H0))
    free.set_state(H, qx, qy, t)
    for _ in range(40):
        assert dyn.step() == free.step()
    for x, y in zip(dyn.state()[:3], free.state()[:3]):
        assert np.array_equal(x, y)
    assert np.abs(dyn.state()[1]).max() > 0.1
    assert abs(dyn.diag()["mass"] - (20 * 10 * 1.0 + 20 * 10 * 0.3)) <= 1e-12 * 260.0


def test_only_walls_on_interior_edges():
    xy, tri, seg = _cut_basin()
    n = len(tri)
    sc = _scenario(xy, tri, seg, np.full(len(seg), 9, np.int32), [S.BC(9, S.OUTFLOW_ZEROGRAD)], np.full(n, 1.0))
    with pytest.raises(oracle.OracleError, match="interior edges"):
        oracle.Sim(sc)
