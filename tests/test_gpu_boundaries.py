"""Standard inflow and outflow conditions on the GPU (section "Hydrodynamic
BCs" and the supplementary feature table: froude inflow, uniform, weir, h-Q
and dynamic-wall outflows): parity with the FP64 oracle (FP64 within 1e-10 of
the norm, FP32 within 1e-4 in the max and L1 norms on a fixed step) on the oracle's
closed-form cases and on wet/dry flows with species, plus argument checks."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import compare, gpu_state, rel_err
from test_oracle_boundaries import _basin_draining, _channel, _flat

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


def _both(sc, swe, t_end, fp32_steps=40):
    st = gpu_state(sc, swe.FP64)
    st.run_until(t_end)
    sim = oracle.Sim(sc)
    sim.run_until(t_end)
    compare(st, sim, FP64_TOL)
    m, d = st.mass(), sim.diag()
    assert abs(m["bnd_flux"] - d["bnd_flux"]) <= FP64_TOL * max(abs(d["bnd_flux"]), 1e-300)
    fixed = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
    st32 = gpu_state(fixed, swe.FP32)
    sim32 = oracle.Sim(fixed)
    for _ in range(fp32_steps):
        st32.step()
        sim32.step()
    compare(st32, sim32, FP32_TOL, metric="l1")
    return st, sim


def test_froude_inflow(swe):
    sc = _channel(60.0, 4.0, 1.0, _flat, 0.0,
                  [S.BC(1, S.INFLOW_FROUDE, slope=2.0, t=np.array([0.0, 2.0]), Q=np.array([1.0, 3.0])),
                   S.BC(2, S.OUTFLOW_ZEROGRAD)], {"x0": 1, "x1": 2})
    st, _ = _both(sc, swe, 4.0)
    assert st.mass()["bnd_flux"] < 0.0


def test_uniform_outflow(swe):
    S0, n, q, hn = 1e-3, 0.03, 0.5, 0.6392264771690853
    sc = _channel(60.0, 4.0, 1.0, lambda x, y: S0 * (60.0 - x), hn,
                  [S.BC(1, S.INFLOW_UNIFORM, slope=S0, t=np.array([0.0]), Q=np.array([2.5 * q * 4.0])),
                   S.BC(2, S.OUTFLOW_UNIFORM, slope=S0)], {"x0": 1, "x1": 2}, manning=n, qx0=q)
    _both(sc, swe, 30.0)


def test_supercritical_uniform_inflow_delivers_exactly_q(swe):
    # the oracle's exact pin, on the GPU: a steep Manning channel with a dry
    # bed takes in exactly Q t through its normal-depth inflow ghost
    Q, S0, n = 2.0, 0.05, 0.01
    sc = _channel(80.0, 4.0, 1.0, lambda x, y: S0 * (80.0 - x), 0.0,
                  [S.BC(1, S.INFLOW_UNIFORM, slope=S0, t=np.array([0.0]), Q=np.array([Q]))], {"x0": 1},
                  manning=n)
    st, _ = _both(sc, swe, 5.0)
    m = st.mass()
    assert m["clipped"] == 0.0
    assert abs(-m["bnd_flux"] - Q * 5.0) <= 1e-12 * Q * 5.0
    assert abs(m["mass"] - Q * 5.0) <= 1e-12 * Q * 5.0
    st32 = gpu_state(sc, swe.FP32)
    st32.run_until(5.0)
    m32 = st32.mass()
    assert abs(-m32["bnd_flux"] - Q * 5.0) <= 1e-6 * Q * 5.0


@pytest.mark.parametrize("kind", ["weir", "hq"])
def test_imposed_outflows(swe, kind):
    bc = (S.BC(2, S.OUTFLOW_WEIR, slope=1.0, par=0.6) if kind == "weir"
          else S.BC(2, S.OUTFLOW_HQ, t=np.array([1.0, 1.2, 2.0]), Q=np.array([0.0, 1.0, 6.0])))
    st, _ = _both(_basin_draining(bc), swe, 30.0)
    assert st.mass()["bnd_flux"] > 0.0


def test_dynamic_wall(swe):
    base = S.dam_break(d=1.0, h_right=0.0)
    xy = base.nodes[:, :2]
    right = np.where(np.abs(xy[:, 0] - 100.0) < 1e-9)[0]
    right = right[np.argsort(xy[right, 1])]
    seg = np.c_[right[:-1], right[1:]].astype(np.int32)
    sc = S.Scenario(**{**base.__dict__, "bnd_seg": seg, "bnd_tag": np.full(len(seg), 7, np.int32),
                       "bcs": [S.BC(7, S.DYNAMIC_WALL, slope=6.0)]})
    st, _ = _both(sc, swe, 10.0)
    assert st.mass()["bnd_flux"] > 0.0


@pytest.mark.parametrize("out", ["uniform", "weir", "hq", "dynwall"])
@pytest.mark.parametrize("seed", range(2))
def test_wet_dry_mixed_with_species(swe, out, seed):
    base = S.tiny_random(6, 4, seed=seed)
    outbc = {"uniform": S.BC(2, S.OUTFLOW_UNIFORM, slope=2e-3),
             "weir": S.BC(2, S.OUTFLOW_WEIR, slope=0.3, par=0.5),
             "hq": S.BC(2, S.OUTFLOW_HQ, t=np.array([0.2, 0.8]), Q=np.array([0.0, 0.5])),
             "dynwall": S.BC(2, S.DYNAMIC_WALL, slope=0.3)}[out]
    r = np.random.default_rng(300 + seed)
    bcs = [S.BC(1, S.INFLOW_FROUDE, slope=0.8, t=np.array([0.0, 1.0]), Q=np.array([0.2, 0.5]), phi_in=(0.9, 0.1)),
           outbc]
    sc = S.Scenario(**{**base.__dict__, "bcs": bcs, "phi0": r.uniform(0, 1, (2, base.n_cells))})
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    for k in range(15):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    compare(st, sim, FP64_TOL)
    q, qo = st.scalars(), sim.scalars()
    for c in range(2):
        assert rel_err(q[c], qo[c]) <= FP64_TOL


def test_argument_checks(swe):
    sc = _basin_draining(S.BC(2, S.OUTFLOW_WEIR, slope=1.0, par=0.0))
    m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    with pytest.raises(swe.SweError, match="Poleni"):
        swe.State(m, sc, precision=swe.FP32)
    bad = _basin_draining(S.BC(2, S.OUTFLOW_HQ, t=np.array([1.0, 2.0]), Q=np.array([0.0, -1.0])))
    with pytest.raises(swe.SweError, match=">= 0"):
        swe.State(m, bad, precision=swe.FP32)
    chezy = S.Scenario(**{**_basin_draining(S.BC(2, S.OUTFLOW_UNIFORM, slope=1e-3)).__dict__,
                          "friction": "chezy", "manning": np.full(sc.n_cells, 0.05)})
    with pytest.raises(swe.SweError, match="Manning or Strickler"):
        swe.State(m, chezy, precision=swe.FP32)
    froude = _basin_draining(S.BC(2, S.INFLOW_FROUDE, slope=0.0, t=np.array([0.0]), Q=np.array([1.0])))
    with pytest.raises(swe.SweError, match="positive"):
        swe.State(m, froude, precision=swe.FP32)
