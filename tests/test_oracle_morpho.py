"""Pins of the Exner module in the oracle (section "Morphodynamics": eq.
exner, eq. exnerupdateformula, the HLL sediment flux eq. exner_hll with the
speeds of eq. exner_wave_assign / eq. exner_wave_estimation, and Table
sedtransport_closure):

* closures: MPM, Grass and Engelund-Hansen magnitudes at chosen Shields
  numbers or speeds, zero below the threshold;
* the derivative dq_B,n/dq_n against a central finite difference of the
  normal transport at fixed depth and tangential velocity;
* the speeds are the roots of lambda^2 - (u_n - c) lambda - D c^2 = 0, one of
  each sign;
* a lake at rest and a flow below the threshold leave the bed bitwise
  unchanged; a closed basin conserves its sediment; with open boundaries and
  a non-erodible bed the volume balance holds to round-off;
* a small hump under a Grass-type transport migrates at the linearised bed
  celerity 3 A u^3 / ((1 - p) h (1 - Fr^2)).
"""
import math

import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M

G = 9.81
K = math.sqrt(1.65 * G * 1e-3 ** 3)


def _cell(closure, alpha, m, thr, h, u, v, cf2, nx=1.0, ny=0.0):
    return oracle.sed_cell(closure, alpha, m, thr, 1e-3, 2.65, G, h, u, v, cf2, nx, ny)


def _cf2_for_theta(theta, U):
    return U * U / (theta * 1.65 * G * 1e-3)


def test_mpm_magnitude_and_threshold():
    U = 1.2
    qbn, D, l1, l2 = _cell("mpm", 8.0, 1.5, 0.047, 0.8, U, 0.0, _cf2_for_theta(0.147, U))
    assert abs(qbn - 8.0 * 0.1 ** 1.5 * K) <= 1e-12 * qbn
    qbn, D, l1, l2 = _cell("mpm", 8.0, 1.5, 0.047, 0.8, U, 0.0, _cf2_for_theta(0.04, U))
    c = math.sqrt(G * 0.8)
    assert qbn == 0.0 and D == 0.0 and l1 == min(0.0, U - c) and l2 == max(0.0, U - c)


def test_grass_and_engelund_hansen_magnitudes():
    qbn, *_ = _cell("grass", 2e-3, 3.0, 0.1, 1.0, 0.0, 1.6, 0.0, nx=0.0, ny=1.0)
    assert abs(qbn - 2e-3 * 1.5 ** 3) <= 1e-15
    U = 0.9
    cf2 = _cf2_for_theta(0.3, U)
    qbn, *_ = _cell("eh", 0.0, 1.0, 0.0, 1.0, U, 0.0, cf2)
    assert abs(qbn - 0.05 * cf2 * 0.3 ** 2.5 * K) <= 1e-12 * qbn


@pytest.mark.parametrize("closure,alpha,m,thr", [("mpm", 8.0, 1.5, 0.047), ("grass", 1e-3, 3.0, 0.05),
                                                 ("eh", 0.0, 1.0, 0.0)])
def test_derivative_matches_finite_difference(closure, alpha, m, thr):
    h, cf2 = 0.7, 300.0
    nx, ny = math.cos(0.4), math.sin(0.4)
    tx, ty = -ny, nx
    un, ut = 1.1, 0.6

    def qbn_at(un_):
        u, v = un_ * nx + ut * tx, un_ * ny + ut * ty
        return _cell(closure, alpha, m, thr, h, u, v, cf2, nx, ny)[0]

    u, v = un * nx + ut * tx, un * ny + ut * ty
    qbn, D, l1, l2 = _cell(closure, alpha, m, thr, h, u, v, cf2, nx, ny)
    dq = 1e-5
    fd = (qbn_at(un + dq / h) - qbn_at(un - dq / h)) / (2 * dq)   # q_n = h u_n
    assert D > 0 and abs(D - fd) <= 1e-6 * abs(D), (D, fd)
    c = math.sqrt(G * h)
    assert l1 <= 0.0 <= l2
    assert abs((l1 + l2) - (un - c)) <= 1e-12
    assert abs(l1 * l2 + D * c * c) <= 1e-12 * max(1.0, D * c * c)


def _box(lx, ly, d, z, H0, morpho, qx0=0.0, **kw):
    xy, tri, _ = M.structured_right(lx, ly, d)
    n = len(tri)
    nodes = np.c_[xy, z(xy[:, 0], xy[:, 1])]
    cx = xy[tri, 0].mean(axis=1)
    H = H0(cx) if callable(H0) else np.full(n, H0)
    base = dict(name="box", nodes=nodes, tri=tri.astype(np.int32), bnd_seg=np.zeros((0, 2), np.int32),
                bnd_tag=np.zeros(0, np.int32), bcs=[], H0=H, h0=None, qx0=np.full(n, qx0), qy0=np.zeros(n),
                manning=np.full(n, 0.025), t_end=10.0, cfl=0.5, morpho=morpho)
    base.update(kw)
    return S.Scenario(**base)


def _bumps(x, y):
    return 0.2 * np.exp(-((x - 10) ** 2 + (y - 5) ** 2) / 8.0) + 0.1 * np.exp(-((x - 25) ** 2 + (y - 3) ** 2) / 5.0)


def test_lake_at_rest_keeps_the_bed():
    sc = _box(30.0, 10.0, 1.0, _bumps, 1.0, S.Morpho("mpm"))
    sim = oracle.Sim(sc)
    z0 = sim.bed()
    for _ in range(200):
        sim.step()
    assert np.array_equal(sim.bed(), z0)
    H, qx, qy, _ = sim.state()
    assert np.all(H == 1.0) and np.all(qx == 0.0) and np.all(qy == 0.0)


def test_flow_below_threshold_keeps_the_bed():
    # a gentle dam break: Shields numbers stay under theta_cr = 0.5
    sc = _box(30.0, 10.0, 1.0, _bumps, lambda x: np.where(x < 15.0, 1.05, 1.0), S.Morpho("mpm", thr=0.5))
    sim = oracle.Sim(sc)
    z0 = sim.bed()
    for _ in range(100):
        sim.step()
    assert np.array_equal(sim.bed(), z0)
    assert np.abs(sim.state()[1]).max() > 0.01


def test_closed_basin_conserves_sediment():
    sc = _box(40.0, 10.0, 1.0, lambda x, y: 0.05 * np.sin(x / 3.0),
              lambda x: np.where(x < 20.0, 1.0, 0.3), S.Morpho("mpm", d_m=1e-3))
    sim = oracle.Sim(sc)
    v0 = sim.morpho_diag()[0]
    z0 = sim.bed()
    m0 = sim.diag()["mass"]
    for _ in range(300):
        sim.step()
    v, b, c = sim.morpho_diag()
    assert b == 0.0 and c == 0.0
    assert np.abs(sim.bed() - z0).max() > 1e-3          # the bed did move
    assert abs(v - v0) <= 1e-12 * abs(v0) + 1e-13
    d = sim.diag()
    assert abs(d["mass"] - (m0 + d["clipped"])) <= 1e-12 * m0   # the depth is kept as the bed moves


def test_open_channel_balance_with_fixed_bed():
    xy, tri, sides = M.structured_right(60.0, 4.0, 1.0)
    n = len(tri)
    segs = [M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), M.segments_on_side(xy, sides["x1"], -1, 1e9, 1)]
    tags = [np.full(len(segs[0]), 1, np.int32), np.full(len(segs[1]), 2, np.int32)]
    z = 0.002 * (60.0 - xy[:, 0])
    # the non-erodible bed 0.2 mm below the initial bed: the scour near the
    # inflow reaches it within the minute
    mo = S.Morpho("mpm", z_rel=np.full(n, -2e-4))
    sc = S.Scenario("open", np.c_[xy, z], tri.astype(np.int32), np.concatenate(segs), np.concatenate(tags),
                    [S.BC(1, S.INFLOW_UNIFORM, slope=2e-3, t=np.array([0.0]), Q=np.array([6.0])),
                     S.BC(2, S.OUTFLOW_ZEROGRAD)], None, np.full(n, 0.5), np.full(n, 1.0), np.zeros(n),
                    np.full(n, 0.02), t_end=60.0, cfl=0.5, morpho=mo)
    sim = oracle.Sim(sc)
    v0 = sim.morpho_diag()[0]
    zfix = sim.bed() - 2e-4
    sim.run_until(60.0)
    v, b, c = sim.morpho_diag()
    assert b != 0.0 and c > 0.0                 # sediment crossed the boundaries, and the fixed bed was reached
    assert np.all(sim.bed() >= zfix)
    assert abs(v - (v0 - b + c)) <= 1e-12 * abs(v0)


def test_hump_migrates_at_the_bed_celerity():
    # frictionless flat channel, uniform inflow at Froude 0.25 (h = 1 m), a
    # 1 cm Gaussian hump; Grass transport q_B = A u^3
    A, p, Fr, h = 5e-3, 0.4, 0.25, 1.0
    u = Fr * math.sqrt(G * h)
    xy, tri, sides = M.structured_right(100.0, 2.0, 0.5)
    n = len(tri)
    segs = [M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), M.segments_on_side(xy, sides["x1"], -1, 1e9, 1)]
    tags = [np.full(len(segs[0]), 1, np.int32), np.full(len(segs[1]), 2, np.int32)]
    bump = lambda x: 0.01 * np.exp(-((x - 30.0) / 4.0) ** 2)   # noqa: E731
    z = bump(xy[:, 0])
    cx = xy[tri, 0].mean(axis=1)
    Q = u * h * 2.0
    mo = S.Morpho("grass", alpha=A, m=3.0, thr=0.0, porosity=p)
    sc = S.Scenario("hump", np.c_[xy, z], tri.astype(np.int32), np.concatenate(segs), np.concatenate(tags),
                    [S.BC(1, S.INFLOW_FROUDE, slope=Fr, t=np.array([0.0]), Q=np.array([Q])),
                     S.BC(2, S.OUTFLOW_ZEROGRAD)], np.full(n, h), None, np.full(n, u * h), np.zeros(n),
                    np.zeros(n), t_end=200.0, cfl=0.5, morpho=mo)
    sim = oracle.Sim(sc)
    area = sim.mesh.geometry()["area"]

    def centre():
        dz = sim.bed() - 0.0
        w = np.clip(dz, 0, None) * area
        sel = (cx > 10.0) & (cx < 90.0)
        return (cx[sel] * w[sel]).sum() / w[sel].sum()

    sim.run_until(20.0)          # the flow settles over the hump
    x0, t0 = centre(), sim.t
    sim.run_until(200.0)
    speed = (centre() - x0) / (sim.t - t0)
    cb = 3.0 * A * u ** 3 / ((1.0 - p) * h * (1.0 - Fr ** 2))
    assert abs(speed - cb) <= 0.05 * cb, (speed, cb)
