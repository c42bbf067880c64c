"""Invariants that pin the oracle: well-balancing (lake at rest, exactly),
conservation, the CFL time step against brute force, the mesh geometry
against direct constructions, rotation invariance, and input validation."""
import math

import numpy as np
import pytest

import oracle
import swe_inputs as S


def test_lake_at_rest_is_exact_over_wet_dry_bed():
    sc = S.lake_at_rest(n_cells=5000, t_end=600.0)
    sim = oracle.Sim(sc)
    H0, _, _, _ = sim.state()
    geo = sim.mesh.geometry()
    dry = H0 - geo["zb"] <= 0
    assert dry.sum() > 50  # islands exist
    m0 = sim.diag()["mass"]
    n = sim.run_until(600.0)
    assert n > 100
    H, qx, qy, t = sim.state()
    assert t == 600.0
    assert np.array_equal(H, H0)
    assert not np.any(qx) and not np.any(qy)
    dg = sim.diag()
    assert dg["mass"] == m0 and dg["clipped"] == 0.0


def test_mass_balance_with_inflow_outflow_and_wet_dry():
    sc = S.valley_flood(n_cells=6000, scale=0.05, t_end=3600.0, q_peak=20.0)
    sim = oracle.Sim(sc)
    m0 = sim.diag()["mass"]
    sim.run_steps(400)
    dg = sim.diag()
    assert dg["bnd_flux"] < 0  # water came in
    inflow = -dg["bnd_flux"]
    assert abs(dg["mass"] - m0 + dg["bnd_flux"] - dg["clipped"]) <= 1e-12 * max(1.0, inflow)


def test_mass_balance_tiny_random_states():
    for seed in range(6):
        sc = S.tiny_random(3, 3, seed=seed)
        sim = oracle.Sim(sc)
        m0 = sim.diag()["mass"]
        sim.run_steps(25)
        dg = sim.diag()
        assert abs(dg["mass"] - m0 + dg["bnd_flux"] - dg["clipped"]) <= 1e-13 * max(1.0, m0)


def _brute_dt(sc, H, qx, qy, zb, t, g=9.81):
    """CFL step from the raw node coordinates: rho = 2 x (distance from the
    centroid to the edge line), lambda = |u.n| + sqrt(g h), wet cells only,
    plus the inflow ghost on its edges."""
    xy = sc.nodes[:, :2]
    best = math.inf
    for i, tri in enumerate(sc.tri):
        h = H[i] - zb[i]
        if not h > sc.h_min:
            continue
        u, v = qx[i] / h, qy[i] / h
        P = xy[tri]
        c = P.mean(axis=0)
        for k in range(3):
            a, b = P[k], P[(k + 1) % 3]
            e = b - a
            nrm = np.array([e[1], -e[0]]) / np.hypot(*e)
            dist = abs(np.dot(c - a, nrm))
            lam = abs(u * nrm[0] + v * nrm[1]) + math.sqrt(g * h)
            best = min(best, 2.0 * dist / lam)
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cfl_step_matches_brute_force(seed):
    sc = S.tiny_random(3, 2, seed=seed, bcs=False)
    sim = oracle.Sim(sc)
    H, qx, qy, t = sim.state()
    zb = sim.mesh.geometry()["zb"]
    dt = sim.next_dt()
    ref = sc.cfl * _brute_dt(sc, H, qx, qy, zb, t)
    assert abs(dt - ref) <= 1e-12 * ref
    # dt_max and t_end caps
    assert sim.next_dt(t_end=t + 0.25 * ref) == pytest.approx(0.25 * ref, rel=1e-15)
    sim2 = oracle.Sim(sc, dt_max=0.5 * ref)
    assert sim2.next_dt() == 0.5 * ref


def test_cfl_step_on_a_moving_lake():
    sc = S.lake_at_rest(n_cells=600, t_end=1.0)
    r = np.random.default_rng(9)
    sc.qx0 = r.uniform(-1, 1, sc.n_cells)
    sc.qy0 = r.uniform(-1, 1, sc.n_cells)
    sim = oracle.Sim(sc)
    H, qx, qy, t = sim.state()
    zb = sim.mesh.geometry()["zb"]
    ref = sc.cfl * _brute_dt(sc, H, qx, qy, zb, t)
    assert abs(sim.next_dt() - ref) <= 1e-12 * ref


def test_inflow_ghost_limits_the_step_of_a_dry_start():
    sc = S.valley_flood(n_cells=3000, scale=0.05)
    sim = oracle.Sim(sc)
    dt = sim.next_dt()
    assert math.isfinite(dt) and 0 < dt < 5.0


def test_geometry_against_direct_constructions():
    sc = S.lake_at_rest(n_cells=2000)
    m = oracle.Mesh(sc.nodes, sc.tri)
    geo = m.geometry()
    N = sc.n_cells
    # Euler: every interior edge has two cells, boundary edges one
    assert 2 * m.n_edges == 3 * N + m.n_boundary_edges
    assert abs(geo["area"].sum() - 2000.0 * 1000.0) < 1e-6
    # closed polygon: sum_k l_k n_k = 0
    s = (geo["length"] * geo["nx"]).sum(1), (geo["length"] * geo["ny"]).sum(1)
    assert np.abs(s[0]).max() < 1e-10 and np.abs(s[1]).max() < 1e-10
    # unit outward normals and rho = 2 x centroid-edge distance
    xy = sc.nodes[:, :2]
    for i in range(0, N, 37):
        P = xy[sc.tri[i]]
        c = P.mean(0)
        for k in range(3):
            n = np.array([geo["nx"][i, k], geo["ny"][i, k]])
            assert abs(np.hypot(*n) - 1) < 1e-14
            # the oracle fixes orientation; find the edge whose normal this is
            dists = []
            for j in range(3):
                a, b = P[j], P[(j + 1) % 3]
                mid = 0.5 * (a + b)
                e = b - a
                if abs(np.dot(e, n)) < 1e-9 * np.hypot(*e):
                    dists.append((abs(np.dot(c - a, n)), np.dot(mid - c, n)))
            assert dists, "normal not perpendicular to any edge"
            d, outward = dists[0]
            assert outward > 0
            assert abs(geo["rho"][i, k] - 2 * d) < 1e-10 * (1 + d)
    # neighbour relation is symmetric
    nbr = geo["nbr"]
    for i in range(0, N, 11):
        for j in nbr[i]:
            if j >= 0:
                assert i in nbr[j]
    # cell bed = mean of node beds
    assert np.allclose(geo["zb"], sc.nodes[sc.tri, 2].mean(1), rtol=0, atol=1e-14)


def _rotate(sc):
    r = S.Scenario(**{**sc.__dict__})
    nodes = sc.nodes.copy()
    nodes[:, 0], nodes[:, 1] = -sc.nodes[:, 1], sc.nodes[:, 0].copy()
    r.nodes = nodes
    r.qx0, r.qy0 = -sc.qy0, sc.qx0.copy()
    return r


@pytest.mark.parametrize("which", ["tiny", "dam"])
def test_rotation_by_90_degrees_is_bitwise(which):
    sc = S.tiny_random(3, 3, seed=4) if which == "tiny" else S.dam_break(1.0)
    a = oracle.Sim(sc)
    b = oracle.Sim(_rotate(sc))
    a.run_steps(15)
    b.run_steps(15)
    Ha, qxa, qya, ta = a.state()
    Hb, qxb, qyb, tb = b.state()
    assert ta == tb
    assert np.array_equal(Ha, Hb)
    assert np.array_equal(qxb, -qya) and np.array_equal(qyb, qxa)


def test_clockwise_input_triangles_are_fixed():
    sc = S.tiny_random(3, 3, seed=2)
    cw = S.Scenario(**{**sc.__dict__})
    t = sc.tri.copy()
    t[:, 1], t[:, 2] = sc.tri[:, 2], sc.tri[:, 1]
    cw.tri = np.ascontiguousarray(t)
    a, b = oracle.Sim(sc), oracle.Sim(cw)
    a.run_steps(10)
    b.run_steps(10)
    assert all(np.array_equal(x, y) for x, y in zip(a.state(), b.state()))


def test_restart_is_bitwise():
    sc = S.tiny_random(3, 3, seed=3)
    a = oracle.Sim(sc)
    a.run_steps(20)
    b = oracle.Sim(sc)
    b.run_steps(8)
    H, qx, qy, t = b.state()
    c = oracle.Sim(sc, t0=t)
    c.set_state(H, qx, qy, t)
    c.run_steps(12)
    assert all(np.array_equal(x, y) for x, y in zip(a.state(), c.state()))


def test_validation_rejects_bad_input():
    sc = S.tiny_random(2, 2, seed=0)
    nodes = sc.nodes.copy()
    # degenerate triangle: collapse one node onto another
    bad = nodes.copy()
    bad[sc.tri[0, 1]] = bad[sc.tri[0, 0]]
    with pytest.raises(oracle.OracleError):
        oracle.Mesh(bad, sc.tri)
    # non-conforming: a third triangle on an existing edge
    tri = np.vstack([sc.tri, sc.tri[:1]])
    with pytest.raises(oracle.OracleError):
        oracle.Mesh(nodes, tri)
    # a tagged segment that is not a boundary edge
    with pytest.raises(oracle.OracleError):
        oracle.Mesh(nodes, sc.tri, np.array([[0, len(nodes) - 1]], np.int32), np.array([1], np.int32))
    for field, value in (("cfl", 1.5), ("cfl", 0.0), ("h_min", 0.0)):
        s2 = S.Scenario(**{**sc.__dict__})
        setattr(s2, field, value)
        with pytest.raises(oracle.OracleError):
            oracle.Sim(s2)
    s2 = S.Scenario(**{**sc.__dict__})
    s2.h0 = sc.h0.copy()
    s2.h0[0] = -0.1
    with pytest.raises(oracle.OracleError):
        oracle.Sim(s2)
    s2.h0[0] = float("nan")
    with pytest.raises(oracle.OracleError):
        oracle.Sim(s2)
