"""Pins of the friction closures (paper: eq. friction_closure with the rows of
Table friction_closure: Strickler, Manning, Chezy, Bezzola) in the oracle.

* Strickler with k_str = 1/n is Manning with n (the two rows define the same
  c_f), over a whole wet/dry run.
* The log-type c_f are continuous where their branches meet (Chezy at
  h = K_s; Bezzola at h/y_R = 2 exactly, and at 0.5 to the printed
  coefficients' precision) and increase with depth.
* A uniform layer on a flat bed, away from the walls, loses discharge exactly
  as the ODE dq/dt = -g h S_f with S_f = u|u| / (g h c_f^2) taken straight
  from eq. friction_closure: the split step is that ODE's exact solution, so
  after any number of steps q = q0 / (1 + q0 t / (h^2 c_f^2)).
"""
import math

import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M

G = 9.81


def _run(sc, steps):
    sim = oracle.Sim(sc)
    for _ in range(steps):
        sim.step()
    return sim.state()


def test_strickler_is_manning_with_inverse_coefficient():
    sc = S.tiny_random(4, 4, seed=3, bcs=False)
    n = np.full(sc.n_cells, 0.03) + 0.02 * (np.arange(sc.n_cells) % 3)
    sc.manning = n
    ref = _run(sc, 20)
    sc2 = S.Scenario(**{**sc.__dict__, "manning": 1.0 / n, "friction": "strickler"})
    got = _run(sc2, 20)
    for a, b in zip(got[:3], ref[:3]):
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(b)))


def test_log_closures_continuous_at_branch_points_and_increasing():
    ks = 0.05
    assert oracle.friction_cf("chezy", ks, ks) == 6.25
    assert abs(oracle.friction_cf("chezy", ks, ks * (1 + 1e-12)) - 6.25) < 1e-10
    yr = 0.2
    at2 = oracle.friction_cf("bezzola", yr, 2 * yr)
    assert abs(oracle.friction_cf("bezzola", yr, 2 * yr * (1 + 1e-12)) - at2) < 1e-9
    # the printed coefficients meet the constant branch to about 0.1 %
    mid = oracle.friction_cf("bezzola", yr, 0.5 * yr)
    assert abs(mid - 1.5) < 2e-3 and oracle.friction_cf("bezzola", yr, 0.5 * yr * (1 - 1e-12)) == 1.5
    for kind, par in (("chezy", ks), ("bezzola", yr)):
        hs = np.geomspace(0.01, 20.0, 400)
        cf = np.array([oracle.friction_cf(kind, par, h) for h in hs])
        assert np.all(np.diff(cf) >= -2e-3), kind


def _strip(n_x=200, n_y=4, dx=0.5):
    xy, tri, _ = M.structured_right(n_x * dx, n_y * dx, dx)
    return xy, tri


@pytest.mark.parametrize("kind,par,h0", [
    ("manning", 0.03, 1.6),
    ("strickler", 30.0, 1.6),
    ("chezy", 0.05, 1.6),
    ("bezzola", 0.16, 1.6),    # h / y_R = 10
    ("bezzola", 1.6, 1.6),     # h / y_R = 1
    ("bezzola", 4.0, 1.6),     # h / y_R < 0.5
])
def test_uniform_layer_decays_as_the_friction_ode(kind, par, h0):
    xy, tri = _strip()
    n = len(tri)
    q0 = 1.2
    sc = S.Scenario("strip", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                    np.zeros(0, np.int32), [], None, np.full(n, h0), np.full(n, q0), np.zeros(n),
                    np.full(n, par), t_end=10.0, friction=kind)
    sc.dt_max = 0.02
    sim = oracle.Sim(sc)
    t = 0.0
    while t < 4.0 - 1e-12:
        t += sim.step()
    H, qx, qy, t_or = sim.state()
    # c_f from the table row, S_f from eq. friction_closure
    if kind == "manning":
        cf = h0 ** (1 / 6) / (par * math.sqrt(G))
    elif kind == "strickler":
        cf = par * h0 ** (1 / 6) / math.sqrt(G)
    elif kind == "chezy":
        cf = 6.25 + math.log(h0 / par) if h0 > par else 6.25
    else:
        r = h0 / par
        cf = (2.5 * math.sqrt(1 - 1 / r) * math.log(10.9 * r) if r > 2 else
              1.25 * math.sqrt(r) * math.log(10.9 * r) if r >= 0.5 else 1.5)
    # dq/dt = -g h S_f(u = q/h) = -(g h / (g h cf^2)) q|q| / h^2
    rate = G * h0 / (G * h0 * cf ** 2) / h0 ** 2
    expect = q0 / (1 + q0 * rate * t_or)
    c = sc.centroids()
    mid = np.abs(c[:, 0] - 50.0) < 5.0    # the walls' waves travel < 25 m by t = 4 s
    assert np.max(np.abs(qx[mid] - expect)) <= 1e-12 * q0, (kind, qx[mid].min(), qx[mid].max(), expect)
    assert np.max(np.abs(H[mid] - h0)) <= 1e-12
    # and friction does something measurable
    assert expect < q0 * 0.995


def test_inflow_needs_a_power_law_closure():
    sc = S.tiny_random(3, 3, seed=1)
    for kind in ("chezy", "bezzola"):
        with pytest.raises(oracle.OracleError, match="Manning or Strickler"):
            oracle.Sim(S.Scenario(**{**sc.__dict__, "friction": kind}))
    oracle.Sim(S.Scenario(**{**sc.__dict__, "manning": 1.0 / sc.manning, "friction": "strickler"}))
