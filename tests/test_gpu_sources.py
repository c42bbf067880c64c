"""External water sources and sinks S_h on the GPU (the S_h paragraph of the
hydrodynamic closure relations, eq. swe_vectorial_form_sourceterms): parity
with the FP64 oracle (FP64 within 1e-10 of the norm, FP32 within 1e-4 in the
L1 norm on a fixed step) for all three modes on wet/dry flows at every tile
size, with and without species; the rain-on-a-basin closed form; the exact
sink's error; the volume balance with the source tally."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M
from gpu_util import compare, gpu_state, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


def _mixed(sc, seed, species=0):
    n = sc.n_cells
    r = np.random.default_rng(200 + seed)
    region = r.integers(-1, 3, n).astype(np.int32)
    srcs = (S.Source(S.SRC_EXACT, S.SRC_DISCHARGE, np.array([0.0, 0.5]), np.array([0.4, -0.05])),
            S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]), np.array([-2.0e4])),
            S.Source(S.SRC_INFINITY))
    kw = {"sources": srcs, "src_region": region}
    if species:
        kw["phi0"] = r.uniform(0.0, 1.0, (species, n))
    return S.Scenario(**{**sc.__dict__, **kw})


def _step_both(st, sim, swe):
    """One step of each; both must fail alike (an exact sink's deficit, which
    ends the run: the GPU state stops stepping).  Returns False then."""
    eg = eo = None
    try:
        dg = st.step()
    except swe.SweError as e:
        eg, dg = e.code, None
    try:
        do = sim.step()
    except oracle.OracleError as e:
        eo, do = e.code, None
    assert (eg is None) == (eo is None), (eg, eo)
    if eg is not None:
        assert eg == swe.ESINK and eo == -8
        return False
    assert abs(dg - do) <= 1e-13 * do, (dg, do)
    return True


@pytest.mark.parametrize("tile", [128, 256, 512])
@pytest.mark.parametrize("seed", range(2))
def test_all_modes_fp64_parity(swe, tile, seed):
    sc = _mixed(S.tiny_random(6, 4, seed=seed), seed)
    st = gpu_state(sc, swe.FP64, block_size=tile)
    sim = oracle.Sim(sc)
    for _ in range(20):
        if not _step_both(st, sim, swe):
            break
    compare(st, sim, FP64_TOL)
    vo = sim.source_volume()
    assert vo != 0.0 and abs(st.source_volume() - vo) <= FP64_TOL * abs(vo)
    m, d = st.mass(), sim.diag()
    assert abs(m["clipped"] - d["clipped"]) <= FP64_TOL * max(abs(d["clipped"]), d["mass"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_tile_with_species(swe, prec):
    sc = _mixed(S.tiny_random(25, 13, seed=6), 6, species=2)
    if prec == "fp32":
        sc = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
    st = gpu_state(sc, swe.FP64 if prec == "fp64" else swe.FP32)
    sim = oracle.Sim(sc)
    for _ in range(25):
        if not _step_both(st, sim, swe):
            break
    q, qo = st.scalars(), sim.scalars()
    if prec == "fp64":
        compare(st, sim, FP64_TOL)
        for c in range(2):
            assert rel_err(q[c], qo[c]) <= FP64_TOL
        vo = sim.source_volume()
        assert abs(st.source_volume() - vo) <= FP64_TOL * abs(vo)
    else:
        compare(st, sim, FP32_TOL, metric="l1")
        area = sim.mesh.geometry()["area"]
        for c in range(2):
            assert (np.abs(q[c] - qo[c]) * area).sum() <= FP32_TOL * (np.abs(qo[c]) * area).sum()
        vo = sim.source_volume()
        assert abs(st.source_volume() - vo) <= 1e-3 * abs(vo)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rain_on_a_closed_basin(swe, prec):
    xy, tri, _ = M.structured_right(20.0, 10.0, 1.0)
    n = len(tri)
    sc = S.Scenario("basin", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                    np.zeros(0, np.int32), [], None, np.full(n, 0.5), np.zeros(n), np.zeros(n),
                    np.full(n, 0.02), t_end=50.0, dt_max=0.5, cfl=0.5,
                    sources=(S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([36.0])),),
                    src_region=np.zeros(n, np.int32))
    st = gpu_state(sc, swe.FP64 if prec == "fp64" else swe.FP32)
    steps = st.run_until(50.0)
    r = st.read()
    assert np.all(r["qx"] == 0.0) and np.all(r["qy"] == 0.0)
    assert np.ptp(r["H"]) == 0.0
    # FP32 keeps the surface as a float plus a 16-bit low part in units of
    # 2^(e-40) for a surface in [2^(e-1), 2^e) (e = 0 here): each step rounds
    # it by at most half of that unit
    tol = 1e-13 if prec == "fp64" else steps * 2.0 ** -41
    assert np.max(np.abs(r["h"] - (0.5 + 1e-5 * 50.0))) <= tol
    assert abs(st.source_volume() - 1e-5 * 50.0 * 200.0) <= (1e-12 if prec == "fp64" else 1e-9) * 200.0


def test_infinity_sink_balance(swe):
    base = S.dam_break(d=1.0, h_right=0.0)
    cx = base.centroids()[:, 0]
    sc = S.Scenario(**{**base.__dict__, "sources": (S.Source(S.SRC_INFINITY),),
                       "src_region": np.where(cx > 80.0, 0, -1).astype(np.int32)})
    st = gpu_state(sc, swe.FP64)
    m0 = st.mass()["mass"]
    st.run_until(8.0)
    sim = oracle.Sim(sc)
    sim.run_until(8.0)
    compare(st, sim, FP64_TOL)
    assert np.all(st.read()["h"][cx > 80.0] == 0.0)
    v = st.source_volume()
    m = st.mass()
    assert v < 0.0 and abs(v - sim.source_volume()) <= FP64_TOL * abs(v)
    assert abs(m["mass"] - (m0 - m["bnd_flux"] + m["clipped"] + v)) <= 1e-12 * m0


def test_exact_sink_deficit_is_reported(swe):
    xy, tri, _ = M.structured_right(4.0, 2.0, 1.0)
    n = len(tri)
    sc = S.Scenario("thin", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                    np.zeros(0, np.int32), [], None, np.full(n, 0.01), np.zeros(n), np.zeros(n),
                    np.zeros(n), t_end=1.0, dt_max=0.5, cfl=0.5,
                    sources=(S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([-3.6e6])),),
                    src_region=np.zeros(n, np.int32))
    st = gpu_state(sc, swe.FP32)
    with pytest.raises(swe.SweError) as e:
        st.step()
    assert e.value.code == swe.ESINK
    assert np.all(st.read()["h"] == 0.0) and st.mass()["clipped"] > 0.0


def test_sources_api(swe):
    sc = S.tiny_random(4, 3, seed=1)
    n = sc.n_cells
    st = gpu_state(sc, swe.FP32, block_size=512)
    assert st.source_volume() == 0.0
    rain = S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([10.0]))
    with pytest.raises(swe.SweError, match="only exact"):
        st.set_sources(np.zeros(n, np.int32), [S.Source(S.SRC_AVAILABLE, S.SRC_INTENSITY, np.array([0.0]),
                                                        np.array([1.0]))])
    with pytest.raises(swe.SweError, match="out of range"):
        st.set_sources(np.full(n, 3, np.int32), [rain])
    with pytest.raises(swe.SweError, match="empty"):
        st.set_sources(np.full(n, -1, np.int32), [S.Source(S.SRC_EXACT, S.SRC_DISCHARGE, np.array([0.0]),
                                                           np.array([1.0]))])
    st.set_sources(np.zeros(n, np.int32), [rain])
    assert st.autotune(2) == 512
    b = swe.Batch(swe.FP32)
    with pytest.raises(swe.SweError, match="not batched"):
        b.add(st, 1.0)
    b.close()
    st.step()
    assert st.source_volume() > 0.0
    st.set_sources(np.zeros(n, np.int32), [])
    assert st.source_volume() == 0.0
    st.step()
