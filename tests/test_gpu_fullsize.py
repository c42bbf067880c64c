"""Parity at the full valley-flood size (4M cells), in the launch
configuration the benchmark times: every output compared with the oracle
after a few steps (the oracle takes about a second per step at this size);
in FP64 also with the draining-time limiter and sources and sinks, with two
passive species, with their diffusion, and with the Exner module; in FP32 also with two species
and with the Exner module (on a fixed step, L1 within 1e-4 and the max
error within the full-size bound); in FP64 with internal conditions on
three bands of interior edges across the valley (a static wall, a rating
curve and a dynamic wall that collapses by depth in the first step)."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import cached, compare, gpu_state, l1_rel, rel_err

pytestmark = pytest.mark.gpu

FULLSIZE_MAX_BOUND = 2e-2


@pytest.fixture(scope="module")
def valley_wet():
    return cached("valley", S.valley_flood, n_cells=4_000_000, snapshot="wet")


@pytest.fixture(scope="module")
def valley_oracle(valley_wet):
    return oracle.Mesh(valley_wet.nodes, valley_wet.tri, valley_wet.bnd_seg, valley_wet.bnd_tag)


def test_fullsize_fp32_three_steps(valley_wet, valley_oracle):
    # FP32 and FP64 states can take different CFL steps (a thin film on one
    # side of the minimum depth changes the global minimum), so the FP32
    # comparison runs with the step fixed just below the CFL limit
    from paper_2102_12862_amd import swe
    sc = S.Scenario(**{**valley_wet.__dict__})
    assert sc.n_cells > 3_900_000
    sc.dt_max = 0.5 * oracle.Sim(sc, mesh=valley_oracle).next_dt()
    st = gpu_state(sc, swe.FP32, block_size=512)
    sim = oracle.Sim(sc, mesh=valley_oracle)
    for _ in range(3):
        st.step()
        sim.step()
    # L1 within 1e-4; the max error, set by the few edges whose reconstructed
    # depth sits within FP32 rounding of zero (see compare), was 8.9e-3
    # (qy) when measured
    errs = compare(st, sim, 1e-4, metric="l1", max_bound=FULLSIZE_MAX_BOUND)
    print("fp32 full size", errs)


def test_fullsize_fp64_two_steps(valley_wet, valley_oracle):
    from paper_2102_12862_amd import swe
    sc = valley_wet
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc, mesh=valley_oracle)
    for _ in range(2):
        st.step()
        sim.step()
    compare(st, sim, 1e-10)


@pytest.mark.parametrize("extra", ["limiter_and_sources", "species", "diffusion", "morpho"])
def test_fullsize_fp64_options(valley_wet, valley_oracle, extra):
    from paper_2102_12862_amd import swe
    n = valley_wet.n_cells
    cx = valley_wet.centroids()[:, 0]
    if extra == "limiter_and_sources":
        # rain on the upper 4 km, a sink of what is there on the lower 4 km
        region = np.where(cx < 4000.0, 0, np.where(cx > 16000.0, 1, -1)).astype(np.int32)
        kw = {"drain": True, "src_region": region,
              "sources": (S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([50.0])),
                          S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]), np.array([-2.0e4])))}
    elif extra in ("species", "diffusion"):
        kw = {"phi0": np.random.default_rng(3).uniform(0.0, 1.0, (2, n))}
        if extra == "diffusion":
            kw["diffusion"] = S.Diffusion(Km=(0.5, 0.05), alpha_L=5.0, alpha_T=0.5, zeta=1.0)
    else:
        kw = {"morpho": S.Morpho("mpm", d_m=1e-3)}
    sc = S.Scenario(**{**valley_wet.__dict__, **kw})
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc, mesh=valley_oracle)
    for _ in range(2):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (dg, do)
    compare(st, sim, 1e-10)
    if extra in ("species", "diffusion"):
        q, qo = st.scalars(), sim.scalars()
        assert all(rel_err(q[c], qo[c]) <= 1e-10 for c in range(2))
    if extra == "morpho":
        assert rel_err(st.bed(), sim.bed()) <= 1e-10


@pytest.mark.parametrize("extra", ["species", "morpho"])
def test_fullsize_fp32_options(valley_wet, valley_oracle, extra):
    from paper_2102_12862_amd import swe
    n = valley_wet.n_cells
    if extra == "species":
        kw = {"phi0": np.random.default_rng(4).uniform(0.0, 1.0, (2, n))}
    else:
        kw = {"morpho": S.Morpho("mpm", d_m=1e-3)}
    sc = S.Scenario(**{**valley_wet.__dict__, **kw})
    sc.dt_max = 0.5 * oracle.Sim(sc, mesh=valley_oracle).next_dt()
    st = gpu_state(sc, swe.FP32)
    sim = oracle.Sim(sc, mesh=valley_oracle)
    for _ in range(3):
        st.step()
        sim.step()
    errs = compare(st, sim, 1e-4, metric="l1", max_bound=FULLSIZE_MAX_BOUND)
    print(f"fp32 full size, {extra}", errs)
    if extra == "species":
        area = valley_oracle.geometry()["area"]
        q, qo = st.scalars(), sim.scalars()
        for c in range(2):
            assert l1_rel(q[c], qo[c], area) <= 1e-4 and rel_err(q[c], qo[c]) <= FULLSIZE_MAX_BOUND
    if extra == "morpho":
        assert rel_err(st.bed(), sim.bed()) <= 1e-4


def _interior_band(sc, x0, half_width=3.0):
    """The interior edges whose midpoints lie within half_width of x = x0, as
    segments running towards +y (so the side left of them is the side
    towards -x)."""
    tri = sc.tri.astype(np.int64)
    xy = sc.nodes[:, :2]
    nn = len(xy) + 1
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = np.minimum(e[:, 0], e[:, 1]) * nn + np.maximum(e[:, 0], e[:, 1])
    u, cnt = np.unique(key, return_counts=True)
    a, b = u[cnt == 2] // nn, u[cnt == 2] % nn
    m = np.abs(0.5 * (xy[a, 0] + xy[b, 0]) - x0) < half_width
    a, b = a[m], b[m]
    up = xy[a, 1] <= xy[b, 1]
    return np.c_[np.where(up, a, b), np.where(up, b, a)].astype(np.int32)


def test_fullsize_fp64_internal_conditions(valley_wet):
    from paper_2102_12862_amd import swe
    bands = [_interior_band(valley_wet, x0) for x0 in (6000.0, 10000.0, 14000.0)]
    assert all(len(bd) > 1000 for bd in bands)
    seg = np.concatenate([valley_wet.bnd_seg] + bands).astype(np.int32)
    tag = np.concatenate([valley_wet.bnd_tag] + [np.full(len(bd), t, np.int32) for bd, t in zip(bands, (9, 10, 11))])
    bcs = list(valley_wet.bcs) + [S.BC(9, S.WALL),
                                  S.BC(10, S.OUTFLOW_HQ, t=np.array([5.0, 15.0]), Q=np.array([0.0, 500.0])),
                                  S.BC(11, S.DYNAMIC_WALL, slope=1e30, par=0.9)]
    sc = S.Scenario(**{**valley_wet.__dict__, "bnd_seg": seg, "bnd_tag": tag, "bcs": bcs})
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    for _ in range(3):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (dg, do)
    compare(st, sim, 1e-10)
