"""Pins of the internal conditions in the oracle (section "Hydrodynamic
BCs": internal static walls, dynamic walls and rating curves on tagged
interior edges):

* a basin cut by a static internal wall evolves, on each side, bitwise like
  that side meshed alone with walls on its cut;
* a dynamic wall stands until its collapse time, then the flow is bitwise
  the flow without the wall restarted from the state at that time;
* a dynamic wall with a collapse depth (the paper's water-depth threshold)
  is bitwise a static wall up to and including the first step that starts
  with a cell next to it at that depth, found by brute force over the
  states, and bitwise the flow without it from then on (inside the domain
  and on its boundary, where the flow without it is zero-gradient outflow);
  a depth never reached keeps it standing;
* an internal rating curve with a linear table drains the upstream half of
  a cut basin (the side left of the cut's segments) into the other half
  along the closed form of A dH/dt = -k (H - H_0), whatever the downstream
  level, the total volume exact and the downstream half gaining what the
  upstream half loses; reversing the segments reverses the flow; the
  species cross with the upstream concentration; a zero table keeps a lake
  at rest bitwise;
* only walls, dynamic walls and rating curves are taken on interior edges,
  and a rating curve refuses the draining-time limiter.
"""
import math

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


def _depth_trigger(make, cells, par, n_after=40, n_max=5000):
    """Steps make("depth") beside make("wall") until the first step that
    started with some cell of `cells` at depth >= par (both bitwise alike
    up to and including it), then beside make("free") restarted from that
    state; returns the time the wall went."""
    dyn, wall = oracle.Sim(make("depth")), oracle.Sim(make("wall"))
    for k in range(n_max):
        h = dyn.state()[0] - dyn.bed()
        fired = bool((h[cells] >= par).any())
        assert dyn.step() == wall.step()
        for x, y in zip(dyn.state()[:3], wall.state()[:3]):
            assert np.array_equal(x, y), k
        if fired:
            break
    else:
        raise AssertionError("the collapse depth was never reached")
    H, qx, qy, t = dyn.state()
    free = oracle.Sim(make("free"))
    free.set_state(H, qx, qy, t)
    for _ in range(n_after):
        assert dyn.step() == free.step()
    for x, y in zip(dyn.state()[:3], free.state()[:3]):
        assert np.array_equal(x, y)
    return t


def _cut_cells(xy, tri, xcut=20.0):
    return np.nonzero((np.abs(xy[tri, 0] - xcut) < 1e-9).sum(axis=1) == 2)[0]


def test_dynamic_wall_collapse_depth_inside():
    xy, tri, seg = _cut_basin()
    cx = xy[tri, 0].mean(axis=1)
    H0 = np.where(cx < 10.0, 1.0, 0.4)
    tags = np.full(len(seg), 9, np.int32)
    bcs = {"depth": [S.BC(9, S.DYNAMIC_WALL, slope=1e30, par=0.6)], "wall": [S.BC(9, S.WALL)], "free": []}
    cells = _cut_cells(xy, tri)
    assert len(cells) == 20
    t = _depth_trigger(lambda k: _scenario(xy, tri, seg, tags, bcs[k], H0), cells, 0.6)
    # the dam-break wave reaches the cut (0.4 m on both sides at the start)
    assert 2.0 < t < 20.0
    # a collapse time before the depth is reached wins
    early = oracle.Sim(_scenario(xy, tri, seg, tags, [S.BC(9, S.DYNAMIC_WALL, slope=1.0, par=0.6)], H0))
    plain = oracle.Sim(_scenario(xy, tri, seg, tags, [S.BC(9, S.DYNAMIC_WALL, slope=1.0)], H0))
    for _ in range(200):
        assert early.step() == plain.step()
    assert np.array_equal(early.state()[0], plain.state()[0])


def test_dynamic_wall_collapse_depth_never_reached():
    xy, tri, seg = _cut_basin()
    cx = xy[tri, 0].mean(axis=1)
    H0 = np.where(cx < 10.0, 1.0, 0.4)
    tags = np.full(len(seg), 9, np.int32)
    dyn = oracle.Sim(_scenario(xy, tri, seg, tags, [S.BC(9, S.DYNAMIC_WALL, slope=1e30, par=5.0)], H0))
    wall = oracle.Sim(_scenario(xy, tri, seg, tags, [S.BC(9, S.WALL)], H0))
    for _ in range(300):
        assert dyn.step() == wall.step()
    for x, y in zip(dyn.state()[:3], wall.state()[:3]):
        assert np.array_equal(x, y)


def test_dynamic_wall_collapse_depth_on_the_boundary():
    base = S.dam_break(d=1.0, h_right=0.0)
    xy = base.nodes[:, :2]
    right = np.where(np.abs(xy[:, 0] - 100.0) < 1e-9)[0]
    right = right[np.argsort(xy[right, 1])]
    seg = np.c_[right[:-1], right[1:]].astype(np.int32)
    bcs = {"depth": [S.BC(7, S.DYNAMIC_WALL, slope=1e30, par=0.05)], "wall": [],
           "free": [S.BC(7, S.OUTFLOW_ZEROGRAD)]}
    def make(k):
        return S.Scenario(**{**base.__dict__, "bnd_seg": seg, "bnd_tag": np.full(len(seg), 7, np.int32),
                             "bcs": bcs[k]})
    cells = np.nonzero((np.abs(base.nodes[base.tri, 0] - 100.0) < 1e-9).sum(axis=1) == 2)[0]
    assert len(cells) > 0
    t = _depth_trigger(make, cells, 0.05)
    assert t > 5.0
    dyn = oracle.Sim(make("depth"))
    dyn.run_until(t)
    assert dyn.diag()["bnd_flux"] == 0.0
    dyn.run_until(t + 5.0)
    assert dyn.diag()["bnd_flux"] > 0.0


def test_dynamic_wall_collapse_depth_must_not_be_negative():
    xy, tri, seg = _cut_basin()
    sc = _scenario(xy, tri, seg, np.full(len(seg), 9, np.int32), [S.BC(9, S.DYNAMIC_WALL, slope=1.0, par=-1.0)],
                   np.full(len(tri), 1.0))
    with pytest.raises(oracle.OracleError, match="collapse depth"):
        oracle.Sim(sc)


def test_only_walls_on_interior_edges():
    xy, tri, seg = _cut_basin()
    n = len(tri)
    sc = _scenario(xy, tri, seg, np.full(len(seg), 9, np.int32), [S.BC(9, S.OUTFLOW_ZEROGRAD)], np.full(n, 1.0))
    with pytest.raises(oracle.OracleError, match="interior edges"):
        oracle.Sim(sc)


K_HQ, H_CREST = 4.0, 1.0


def _rating_basin(reverse=False, H_up=1.3, H_down=0.5, k=K_HQ, phi=False):
    """The 40 m x 10 m basin cut at x = 20 by a rating curve Q(H) = k (H - 1)
    (0 below H = 1); the cut's segments run along +y, so the half x < 20
    lies on their left (upstream), or along -y with reverse."""
    xy, tri, seg = _cut_basin()
    if reverse:
        seg = seg[:, ::-1].copy()
    cx = xy[tri, 0].mean(axis=1)
    left = cx < 20.0
    up = ~left if reverse else left
    H0 = np.where(up, H_up, H_down)
    bc = S.BC(9, S.OUTFLOW_HQ, t=np.array([H_CREST, H_CREST + 1.0]), Q=np.array([0.0, k]))
    sc = _scenario(xy, tri, seg, np.full(len(seg), 9, np.int32), [bc], H0)
    sc.dt_max = 0.5
    if phi:
        sc.phi0 = np.where(up, 1.0, 0.0)[None, :]
    return sc, up


@pytest.mark.parametrize("reverse", [False, True])
def test_rating_curve_drains_the_upstream_half(reverse):
    sc, up = _rating_basin(reverse)
    sim = oracle.Sim(sc)
    area = sim.mesh.geometry()["area"]
    a_up = area[up].sum()
    v0 = sim.diag()["mass"]
    vu0 = ((sim.state()[0] - sim.bed()) * area)[up].sum()
    T = 200.0
    sim.run_until(T)
    H = sim.state()[0]
    h = H - sim.bed()
    # A dH/dt = -k (H - 1) over the upstream half (its level stays near flat)
    expect = H_CREST + (1.3 - H_CREST) * math.exp(-K_HQ * T / a_up)
    mean_up = (H[up] * area[up]).sum() / a_up
    assert abs(mean_up - expect) <= 0.02 * (expect - H_CREST), (mean_up, expect)
    # the total exact, the downstream half gains what the upstream half lost
    d = sim.diag()
    assert d["bnd_flux"] == 0.0 and d["clipped"] == 0.0
    assert abs(d["mass"] - v0) <= 1e-12 * v0
    vu = (h * area)[up].sum()
    vd = (h * area)[~up].sum()
    assert abs((vu0 - vu) - (vd - (v0 - vu0))) <= 1e-11 * v0
    assert vu0 - vu > 0.5 * (1.3 - expect) * a_up


def test_rating_curve_is_one_way():
    # the downstream half higher than the upstream one: the curve still
    # passes Q(H_upstream) downstream, and nothing flows back
    sc, up = _rating_basin(H_up=1.2, H_down=1.6)
    sim = oracle.Sim(sc)
    area = sim.mesh.geometry()["area"]
    vu0 = ((sim.state()[0] - sim.bed()) * area)[up].sum()
    sim.run_until(50.0)
    vu = ((sim.state()[0] - sim.bed()) * area)[up].sum()
    assert vu < vu0


def test_rating_curve_carries_the_upstream_concentration():
    sc, up = _rating_basin(phi=True)
    sim = oracle.Sim(sc)
    area = sim.mesh.geometry()["area"]
    vd0 = ((sim.state()[0] - sim.bed()) * area)[~up].sum()
    sim.run_until(100.0)
    vd = ((sim.state()[0] - sim.bed()) * area)[~up].sum()
    q = sim.scalars()[0]
    # the upstream half stays at phi = 1; what entered downstream is exactly
    # the water that crossed, at phi = 1
    assert abs((q * area)[~up].sum() - (vd - vd0)) <= 1e-10 * (vd - vd0)
    m, b, c = sim.scalar_diag()
    assert b[0] == 0.0 and abs(m[0] - ((1.3 - 0.0) * area[up].sum())) <= 1e-11 * m[0]


def test_zero_rating_curve_keeps_a_lake_at_rest():
    sc, _ = _rating_basin(H_up=1.4, H_down=1.4, k=0.0)
    sim = oracle.Sim(sc)
    H0 = sim.state()[0].copy()
    for _ in range(100):
        sim.step()
    H, qx, qy, _ = sim.state()
    assert np.array_equal(H, H0) and np.all(qx == 0.0) and np.all(qy == 0.0)


def test_rating_curve_refuses_the_limiter():
    sc, _ = _rating_basin()
    sim = oracle.Sim(sc)
    with pytest.raises(oracle.OracleError, match="do not combine"):
        sim.set_drain(True)
