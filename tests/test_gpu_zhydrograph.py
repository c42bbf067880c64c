"""Prescribed water-surface boundary ("zhydrograph") on the GPU: parity with
the FP64 oracle while a basin fills and drains through it, a lake at the
boundary's level staying exactly at rest, and the volume balance."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import compare, gpu_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


@pytest.mark.parametrize("levels,H0", [([0.3, 0.9], 0.3), ([0.9, 0.4], 0.9)])
def test_fill_and_drain_parity_fp64(swe, levels, H0):
    sc = S.level_basin([0.0, 20.0], levels, H0=H0, t_end=60.0)
    st = gpu_state(sc, swe.FP64)
    st.run_until(30.0)
    sim = oracle.Sim(sc)
    sim.run_until(30.0)
    compare(st, sim, 1e-10)
    m = st.mass()
    d = sim.diag()
    assert abs(m["bnd_flux"] - d["bnd_flux"]) <= 1e-10 * abs(d["bnd_flux"])


def test_fill_parity_fp32_fixed_step(swe):
    sc = S.level_basin([0.0, 20.0], [0.3, 0.9], H0=0.3, t_end=60.0)
    sc.dt_max = 0.5 * oracle.Sim(sc).next_dt()
    st = gpu_state(sc, swe.FP32)
    sim = oracle.Sim(sc)
    for _ in range(200):
        st.step()
        sim.step()
    compare(st, sim, 1e-4, metric="l1")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lake_at_boundary_level_exact(swe, prec):
    sc = S.level_basin([0.0], [0.625], H0=0.625)
    st = gpu_state(sc, swe.FP64 if prec == "fp64" else swe.FP32)
    r0 = st.read()
    for _ in range(100):
        st.step()
    r = st.read()
    assert np.array_equal(r["H"], r0["H"]) and not r["qx"].any() and not r["qy"].any()
