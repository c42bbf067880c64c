"""Friction closures of Table friction_closure (Manning, Strickler, Chezy,
Bezzola) on the GPU: parity with the FP64 oracle in both precisions, the
uniform-layer decay against the closed form of the split friction ODE, and
the inflow restriction to power-law closures."""
import math

import numpy as np
import pytest

import oracle
import swe_inputs as S
from gpu_util import compare, gpu_state
from swe_inputs import mesh as M

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4
CLOSURES = [("manning", 0.03), ("strickler", 25.0), ("chezy", 0.02), ("bezzola", 0.15)]


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


def _no_inflow(sc, kind, par):
    n = sc.n_cells
    rng = np.random.default_rng(7)
    p = par * rng.uniform(0.5, 1.5, n)
    p[rng.random(n) < 0.1] = 0.0  # some frictionless cells
    return S.Scenario(**{**sc.__dict__, "bcs": [b for b in sc.bcs if b.kind != S.INFLOW_UNIFORM],
                         "manning": p, "friction": kind})


@pytest.mark.parametrize("kind,par", CLOSURES)
@pytest.mark.parametrize("seed", range(3))
def test_tiny_wet_dry_fp64(swe, kind, par, seed):
    sc = _no_inflow(S.tiny_random(4, 3, seed=seed), kind, par)
    st = gpu_state(sc, swe.FP64)
    sim = oracle.Sim(sc)
    for k in range(10):
        dg, do = st.step(), sim.step()
        assert abs(dg - do) <= 1e-13 * do, (k, dg, do)
    compare(st, sim, FP64_TOL)


@pytest.mark.parametrize("kind,par", CLOSURES)
def test_dam_break_with_friction_both_precisions(swe, kind, par):
    base = S.dam_break(d=1.0, h_right=0.0)   # Ritter set-up: a wet/dry front
    sc = S.Scenario(**{**base.__dict__, "manning": np.full(base.n_cells, par), "friction": kind, "t_end": 1.0})
    st = gpu_state(sc, swe.FP64)
    st.run_until(1.0)
    sim = oracle.Sim(sc)
    sim.run_until(1.0)
    compare(st, sim, FP64_TOL)
    # FP32 on a fixed step (the CFL step would follow FP32 rounding)
    fixed = S.Scenario(**{**sc.__dict__, "dt_max": 0.5 * oracle.Sim(sc).next_dt()})
    st32 = gpu_state(fixed, swe.FP32)
    sim32 = oracle.Sim(fixed)
    for _ in range(40):
        st32.step()
        sim32.step()
    compare(st32, sim32, FP32_TOL, metric="l1")


@pytest.mark.parametrize("kind,par", CLOSURES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_layer_decay_closed_form(swe, kind, par, prec):
    xy, tri, _ = M.structured_right(100.0, 2.0, 0.5)
    n = len(tri)
    h0, q0 = 1.6, 1.2
    sc = S.Scenario("strip", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                    np.zeros(0, np.int32), [], None, np.full(n, h0), np.full(n, q0), np.zeros(n),
                    np.full(n, par), t_end=4.0, dt_max=0.02, friction=kind)
    st = gpu_state(sc, swe.FP64 if prec == "fp64" else swe.FP32)
    st.run_until(4.0)
    r = st.read()
    cf = {"manning": lambda: h0 ** (1 / 6) / (par * math.sqrt(9.81)),
          "strickler": lambda: par * h0 ** (1 / 6) / math.sqrt(9.81),
          "chezy": lambda: 6.25 + math.log(h0 / par),
          "bezzola": lambda: 2.5 * math.sqrt(1 - par / h0) * math.log(10.9 * h0 / par)}[kind]()
    expect = q0 / (1 + q0 * 4.0 / (h0 ** 2 * cf ** 2))
    mid = np.abs(sc.centroids()[:, 0] - 50.0) < 5.0
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert np.max(np.abs(r["qx"][mid] - expect)) <= tol * q0, (r["qx"][mid].min(), r["qx"][mid].max(), expect)


def test_inflow_needs_a_power_law_closure(swe):
    sc = S.tiny_random(3, 3, seed=2)
    m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
    for kind in ("chezy", "bezzola"):
        with pytest.raises(swe.SweError, match="Manning or Strickler"):
            swe.State(m, S.Scenario(**{**sc.__dict__, "friction": kind}), precision=swe.FP32)
    st = swe.State(m, S.Scenario(**{**sc.__dict__, "manning": 1.0 / sc.manning, "friction": "strickler"}),
                   precision=swe.FP64)
    st.step()
