"""Pins of the passive-scalar module in the oracle (section "Scalar
advection-diffusion": eq. scalar_goveq and eq. scl:updateformula with the
advective fluxes; benchmarks T5 and T6).

* T5: two rarefactions leave the scalar contact at x = 50 m in place; the
  concentration stays 1 on the left and 0 on the right (paper: the contact is
  perfectly maintained), to round-off.
* T6: the initial species masses over the initial water volume give the
  resting concentrations the paper prints (0.386 and 0.023), which pins the
  reading of its initial conditions; over a long run the species masses are
  conserved with walls and the concentrations stay within their initial
  bounds (upwind advection is monotone).
* A uniform concentration stays uniform in any flow (the scalar update is
  the water update times the concentration).
"""
import numpy as np

import oracle
import swe_inputs as S


def _phi(sim, sc):
    q = sim.scalars()
    H = sim.state()[0]
    zb = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag).geometry()["zb"]
    h = H - zb
    return np.where(h > 0, q / np.where(h > 0, h, 1.0), 0.0), h


def test_t5_contact_is_kept():
    sc = S.t5_rarefactions(d=0.1)
    sim = oracle.Sim(sc)
    sim.run_until(2.5)
    phi, h = _phi(sim, sc)
    cx = sc.centroids()[:, 0]
    assert h.min() > 0.2   # the depression stays wet (h* = 0.2715 m)
    assert np.max(np.abs(phi[0, cx < 50.0] - 1.0)) <= 1e-12
    assert np.max(np.abs(phi[0, cx > 50.0])) <= 1e-12


def test_t6_resting_concentrations():
    # on an 80k-cell mesh the cell discretisation of the initial condition is
    # below the printed rounding
    sc = S.t6_three_humps(n_cells=80000)
    sim = oracle.Sim(sc)
    m0, _, _ = sim.scalar_diag()
    v0 = sim.diag()["mass"]
    assert abs(m0[0] / v0 - 0.386) < 6e-4 and abs(m0[1] / v0 - 0.023) < 6e-4, (m0 / v0)


def test_t6_species_mass_conserved_and_bounded():
    sc = S.t6_three_humps(n_cells=4000)
    sim = oracle.Sim(sc)
    m0, _, _ = sim.scalar_diag()
    steps = 1500
    for _ in range(steps):
        sim.step()
    m, b, c = sim.scalar_diag()
    assert np.all(b == 0.0)
    assert np.all(np.abs(m - (m0 + c)) <= 100 * np.finfo(float).eps * steps * m0), (m - m0, c)
    assert np.all(np.abs(c) <= 1e-3 * m0)   # the reset moves little mass
    phi, h = _phi(sim, sc)
    wet = h > 1e-3
    assert phi[0, wet].min() >= -1e-12 and phi[0, wet].max() <= 0.5 + 1e-12
    assert phi[1, wet].min() >= -1e-12 and phi[1, wet].max() <= 0.1 + 1e-12


def test_uniform_concentration_stays_uniform():
    sc = S.tiny_random(4, 4, seed=2, bcs=False)
    n = sc.n_cells
    sim = oracle.Sim(S.Scenario(**{**sc.__dict__, "phi0": np.full((1, n), 0.3)}))
    for _ in range(20):
        sim.step()
    phi, h = _phi(sim, sc)
    wet = h > 0
    assert np.max(np.abs(phi[0, wet] - 0.3)) <= 1e-12
