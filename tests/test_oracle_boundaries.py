"""Pins of the standard inflow and outflow conditions beyond uniform inflow,
zero gradient and zhydrograph (section "Hydrodynamic BCs" and the
supplementary feature table: froude inflow, uniform, weir, h-Q relation and
dynamic-wall outflows), against closed forms:

* an inflow imposes its discharge: a uniform or Froude inflow delivers
  exactly the hydrograph's volume, sum over steps of Q(t^n) dt, whether its
  boundary state is subcritical (a mild channel filling a basin, a rising
  hydrograph) or supercritical (a Froude inflow onto a dry bed, a steep
  channel), and the inflowing layer carries the boundary depth
  (q / (Fr sqrt(g)))^(2/3) or the normal depth in the supercritical case;
* a uniform outflow keeps uniform (normal) flow down a Manning channel;
* a basin draining over a Poleni weir follows the closed form of
  dV/dt = -(2/3) mu sqrt(2g) (H - z_w)^(3/2) L;
* a basin draining through a linear h-Q relation decays exponentially;
* a dynamic wall is a wall bitwise until its collapse time, then open.
"""
import math

import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M

G = 9.81


def _channel(lx, ly, d, z, h0, bcs, side_tags, manning=0.0, qx0=0.0, **kw):
    """Rectangle with tagged sides (x0 / x1 -> tag), bed z(x, y)."""
    xy, tri, sides = M.structured_right(lx, ly, d)
    n = len(tri)
    segs, tags = [], []
    for side, tag in side_tags.items():
        s = M.segments_on_side(xy, sides[side], -1, 1e9, 1 if side in ("x0", "x1") else 0)
        segs.append(s)
        tags.append(np.full(len(s), tag, np.int32))
    nodes = np.c_[xy, z(xy[:, 0], xy[:, 1])]
    base = dict(name="channel", nodes=nodes, tri=tri.astype(np.int32),
                bnd_seg=np.concatenate(segs) if segs else np.zeros((0, 2), np.int32),
                bnd_tag=np.concatenate(tags) if tags else np.zeros(0, np.int32), bcs=bcs, H0=None,
                h0=np.full(n, h0) if np.isscalar(h0) else h0, qx0=np.full(n, qx0), qy0=np.zeros(n),
                manning=np.full(n, manning), t_end=100.0, cfl=0.5)
    base.update(kw)
    return S.Scenario(**base)


def _flat(x, y):
    return np.zeros_like(x)


def test_supercritical_froude_inflow_onto_a_dry_bed():
    Q, Fr, ly = 2.0, 2.0, 4.0
    sc = _channel(60.0, ly, 1.0, _flat, 0.0,
                  [S.BC(1, S.INFLOW_FROUDE, slope=Fr, t=np.array([0.0]), Q=np.array([Q])),
                   S.BC(2, S.OUTFLOW_ZEROGRAD)], {"x0": 1, "x1": 2})
    sim = oracle.Sim(sc)
    sim.run_until(4.0)
    d = sim.diag()
    assert d["bnd_flux"] < 0
    assert abs(-d["bnd_flux"] - Q * 4.0) <= 1e-12 * Q * 4.0
    assert abs(d["mass"] - Q * 4.0) <= 1e-12 * Q * 4.0
    q = Q / ly
    hg = (q / (Fr * math.sqrt(G))) ** (2.0 / 3.0)
    H, qx, qy, _ = sim.state()
    cx = sc.centroids()[:, 0]
    near = cx < 3.0
    assert np.max(np.abs(H[near] - hg)) <= 0.02 * hg
    assert np.max(np.abs(qx[near] - q)) <= 0.02 * q


def test_supercritical_uniform_inflow_delivers_exactly_q():
    # a steep Manning channel: the normal-depth ghost (n q / sqrt(S))^(3/5) is
    # supercritical, so on a dry bed every wave of the inflow edge points into
    # the domain and the edge flux is the ghost's own: exactly Q t enters
    Q, S0, n, ly = 2.0, 0.05, 0.01, 4.0
    q = Q / ly
    hn = (n * q / math.sqrt(S0)) ** 0.6
    assert q / hn > 2.0 * math.sqrt(G * hn)  # Froude number above 2
    sc = _channel(80.0, ly, 1.0, lambda x, y: S0 * (80.0 - x), 0.0,
                  [S.BC(1, S.INFLOW_UNIFORM, slope=S0, t=np.array([0.0]), Q=np.array([Q]))], {"x0": 1},
                  manning=n)
    sim = oracle.Sim(sc)
    sim.run_until(5.0)
    d = sim.diag()
    assert d["clipped"] == 0.0
    assert abs(-d["bnd_flux"] - Q * 5.0) <= 1e-12 * Q * 5.0
    assert abs(d["mass"] - Q * 5.0) <= 1e-12 * Q * 5.0
    # the layer next to the inlet carries about the normal depth and
    # discharge (on a 5 % slope the first-order scheme's own equilibrium
    # differs from the continuous normal flow by a few per cent)
    H, qx, _, _ = sim.state()
    h = H - sim.mesh.geometry()["zb"]
    near = sc.centroids()[:, 0] < 3.0
    assert np.max(np.abs(h[near] - hn)) <= 0.1 * hn
    assert np.max(np.abs(qx[near] - q)) <= 0.1 * q


def _hydrograph_volume(sim, Q, t_end):
    """Runs to t_end and returns sum over steps of Q(t^n) dt_n, the volume
    an inflow that imposes its discharge delivers (hydrograph at t^n)."""
    parts = []
    while sim.t < t_end:
        t0 = sim.t
        parts.append(Q(t0) * sim.step(t_end))
    return math.fsum(parts)


@pytest.mark.parametrize("kind", ["uniform", "froude"])
def test_subcritical_inflow_delivers_the_hydrograph_volume(kind):
    # a mild channel (slope 1e-3) filling a closed basin through a rising
    # hydrograph: the boundary state is subcritical (Froude 0.5 for the
    # froude inflow, about 0.2 at the normal depth), so waves leave the
    # domain through the inlet, and still exactly the hydrograph enters
    ly = 4.0
    ts, Qs = np.array([0.0, 20.0]), np.array([0.5, 2.5])

    def Q(t):
        return float(np.interp(t, ts, Qs))

    if kind == "uniform":
        bc = S.BC(1, S.INFLOW_UNIFORM, slope=1e-3, t=ts, Q=Qs)
        q = Qs[-1] / ly
        hn = (0.03 * q / math.sqrt(1e-3)) ** 0.6
        assert q / hn < 0.5 * math.sqrt(G * hn)
    else:
        bc = S.BC(1, S.INFLOW_FROUDE, slope=0.5, t=ts, Q=Qs)
    sc = _channel(40.0, ly, 1.0, lambda x, y: 1e-3 * (40.0 - x), 0.3, [bc], {"x0": 1}, manning=0.03)
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    vol = _hydrograph_volume(sim, Q, 20.0)
    d = sim.diag()
    assert abs(-d["bnd_flux"] - vol) <= 1e-13 * vol
    assert abs(d["mass"] - m0 - vol) <= 1e-12 * d["mass"]
    # and the discrete volume is the hydrograph's integral up to O(dt)
    assert abs(vol - 30.0) <= 0.01 * 30.0


def test_uniform_outflow_keeps_normal_flow():
    S0, n, q, ly = 1e-3, 0.03, 0.5, 4.0
    hn = (n * q / math.sqrt(S0)) ** 0.6
    sc = _channel(200.0, ly, 1.0, lambda x, y: S0 * (200.0 - x), hn,
                  [S.BC(1, S.INFLOW_UNIFORM, slope=S0, t=np.array([0.0]), Q=np.array([q * ly])),
                   S.BC(2, S.OUTFLOW_UNIFORM, slope=S0)], {"x0": 1, "x1": 2}, manning=n, qx0=q)
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    sim.run_until(300.0)
    H, qx, _, _ = sim.state()
    zb = sim.mesh.geometry()["zb"]
    h = H - zb
    assert np.max(np.abs(h - hn)) <= 5e-3 * hn, (h.min(), h.max(), hn)
    assert np.max(np.abs(qx - q)) <= 5e-3 * q
    d = sim.diag()
    assert abs(d["mass"] - (m0 - d["bnd_flux"] + d["clipped"])) <= 1e-12 * m0


def test_uniform_outflow_needs_a_power_law_closure():
    sc = _channel(10.0, 2.0, 1.0, _flat, 0.5, [S.BC(2, S.OUTFLOW_UNIFORM, slope=1e-3)], {"x1": 2},
                  manning=5.0, friction="chezy")
    with pytest.raises(oracle.OracleError, match="Manning or Strickler"):
        oracle.Sim(sc)


def _basin_draining(bc, lx=40.0, ly=20.0, H0=1.3):
    # the outflow takes the whole x = lx side
    return _channel(lx, ly, 1.0, _flat, H0, [bc], {"x1": 2}, dt_max=0.5)


def test_weir_drains_a_basin_by_poleni():
    mu, zw, H0, lx, ly = 0.6, 1.0, 1.3, 40.0, 20.0
    sc = _basin_draining(S.BC(2, S.OUTFLOW_WEIR, slope=zw, par=mu), lx, ly, H0)
    sim = oracle.Sim(sc)
    T = 200.0
    sim.run_until(T)
    H = sim.state()[0]
    # dH/dt = -K (H - zw)^(3/2), K = (2/3) mu sqrt(2g) L / A
    K = (2.0 / 3.0) * mu * math.sqrt(2 * G) * ly / (lx * ly)
    expect = zw + ((H0 - zw) ** -0.5 + 0.5 * K * T) ** -2.0
    mean = H.mean()
    assert abs((mean - zw) - (expect - zw)) <= 0.02 * (expect - zw), (mean, expect)
    d = sim.diag()
    assert abs(d["mass"] - (H0 * lx * ly - d["bnd_flux"] + d["clipped"])) <= 1e-12 * H0 * lx * ly


def test_weir_below_crest_is_a_wall():
    sc = _basin_draining(S.BC(2, S.OUTFLOW_WEIR, slope=1.5, par=0.6))
    sim = oracle.Sim(sc)
    sim.run_until(20.0)
    H, qx, qy, _ = sim.state()
    assert np.all(H == 1.3) and np.all(qx == 0.0) and np.all(qy == 0.0)
    assert sim.diag()["bnd_flux"] == 0.0


def test_linear_hq_relation_drains_exponentially():
    lx, ly, H0, k = 40.0, 20.0, 1.3, 4.0
    # Q(H) = k (H - 1) over the side, 0 below H = 1
    bc = S.BC(2, S.OUTFLOW_HQ, t=np.array([1.0, 2.0]), Q=np.array([0.0, k]))
    sim = oracle.Sim(_basin_draining(bc, lx, ly, H0))
    T = 300.0
    sim.run_until(T)
    expect = 1.0 + (H0 - 1.0) * math.exp(-k * T / (lx * ly))
    assert abs(sim.state()[0].mean() - expect) <= 0.02 * (expect - 1.0)


def test_hq_relation_rejects_negative_discharge():
    bc = S.BC(2, S.OUTFLOW_HQ, t=np.array([1.0, 2.0]), Q=np.array([0.0, -1.0]))
    with pytest.raises(oracle.OracleError, match=">= 0"):
        oracle.Sim(_basin_draining(bc))


def test_dynamic_wall_collapses_at_its_time():
    base = S.dam_break(d=1.0, h_right=0.0)
    xy = base.nodes[:, :2]
    right = np.where(np.abs(xy[:, 0] - 100.0) < 1e-9)[0]
    right = right[np.argsort(xy[right, 1])]
    seg = np.c_[right[:-1], right[1:]].astype(np.int32)
    def sc_with(bcs):
        return S.Scenario(**{**base.__dict__, "bnd_seg": seg, "bnd_tag": np.full(len(seg), 7, np.int32),
                             "bcs": bcs})
    wall = oracle.Sim(sc_with([]))
    dyn = oracle.Sim(sc_with([S.BC(7, S.DYNAMIC_WALL, slope=6.0)]))
    while wall.t < 6.0:
        assert wall.step() == dyn.step()
    for a, b in zip(wall.state()[:3], dyn.state()[:3]):
        assert np.array_equal(a, b)
    assert dyn.diag()["bnd_flux"] == 0.0
    dyn.run_until(10.0)
    wall.run_until(10.0)
    assert dyn.diag()["bnd_flux"] > 0.0 and wall.diag()["bnd_flux"] == 0.0
