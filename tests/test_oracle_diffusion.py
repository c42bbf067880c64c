"""Pins of the species diffusion in the oracle (section "Scalar advection-
diffusion": the Cattaneo-type relaxation of eq. relaxation_terms, the
relaxed flux of eq. vecform_scalar2 solved at each edge as a two-wave
Riemann problem, the update of eq. scl:updateformula with the stiff
relaxation source by the locally implicit Euler step; the dispersion closure
of section "Scalar advection-diffusion closure relationships"):

* a Gaussian in water at rest spreads like the heat equation's closed form,
  and the error falls as the mesh is refined with the relaxation time tied to
  the mesh (zeta = 1 s/m times the leg), the species mass exact throughout;
* the T6 dam break over three humps mixes its two species to the uniform
  concentrations of its species mass over its water volume (the printed
  fully mixed 0.386 / 0.023 on the fine mesh), which advection alone never
  reaches;
* a uniform concentration stays uniform, with the auxiliary variables at
  zero, in flowing water over a varying bed;
* turbulent dispersion spreads a patch along a uniform flow faster than
  across it, by about the ratio alpha_L / alpha_T of the closure.
"""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M

K = 0.25


def _strip(d, phi0, psi0, zeta, t_end):
    xy, tri, _ = M.structured_right(10.0, 2 * d, d)
    n = len(tri)
    sc = S.Scenario("strip", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                    np.zeros(0, np.int32), [], None, np.ones(n), np.zeros(n), np.zeros(n), np.zeros(n),
                    t_end=t_end, cfl=0.5, phi0=phi0(xy[tri].mean(axis=1)[:, 0])[None, :])
    sim = oracle.Sim(sc)
    cx = xy[tri].mean(axis=1)[:, 0]
    sim.set_diffusion(S.Diffusion(Km=K, zeta=zeta), psi0=np.stack([psi0(cx), np.zeros(n)], axis=1)[None])
    return sim, cx


def test_gaussian_spreads_like_the_heat_equation():
    # phi(x, t) = sqrt(t0 / (t0 + t)) exp(-(x - 5)^2 / (4 K (t0 + t))); walls
    # are far outside the Gaussian; CFL 0.5 on right triangles (the printed
    # step is unstable above about 0.6 there)
    t0, T = 0.5, 1.0

    def exact(x, t):
        return np.sqrt(t0 / (t0 + t)) * np.exp(-(x - 5.0) ** 2 / (4 * K * (t0 + t)))

    errs = []
    for d in (0.2, 0.1, 0.05, 0.025):
        sim, cx = _strip(d, lambda x: exact(x, 0.0), lambda x: -2 * (x - 5.0) / (4 * K * t0) * exact(x, 0.0),
                         zeta=1.0 * d, t_end=T)
        m0 = sim.scalar_diag()[0][0]
        sim.run_until(T)
        q = sim.scalars()[0]
        errs.append(np.abs(q - exact(cx, T)).max())
        assert abs(sim.scalar_diag()[0][0] - m0) <= 1e-14 * m0
    # converging (about d^(1/2): numerical diffusion sqrt(K/zeta) d / 2 with
    # zeta proportional to d), and close on the finest mesh
    assert all(b < 0.75 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.05 * exact(5.0, T), errs
    # without diffusion the Gaussian would keep its initial peak
    assert exact(5.0, 0.0) - exact(5.0, T) > 10 * errs[-1]


def _t6(diffusion, n_cells=5000, t_end=1200.0):
    sc = S.t6_three_humps(n_cells, t_end=t_end)
    if diffusion:
        sc.diffusion = S.Diffusion(Km=25.0, zeta=10.0)
    return sc


@pytest.mark.parametrize("diffusion", [True, False])
def test_t6_mixes_to_the_fully_mixed_concentrations(diffusion):
    # a large diffusivity (25 m^2/s) mixes the basin within minutes; the
    # relaxation waves sqrt(K / zeta) stay below the water's celerity
    sc = _t6(diffusion)
    sim = oracle.Sim(sc)
    m0 = sim.scalar_diag()[0]
    sim.run_until(sc.t_end)
    m, b, c = sim.scalar_diag()
    assert np.all(np.abs(m - m0 - c) <= 1e-12 * m0) and np.all(b == 0.0)
    H, _, _, _ = sim.state()
    h = H - sim.bed()
    area = sim.mesh.geometry()["area"]
    mixed = m / (h * area).sum()
    wet = h > 0.01
    phi = sim.scalars()[:, wet] / h[wet]
    spread = (phi.max(axis=1) - phi.min(axis=1)) / mixed
    if diffusion:
        assert np.all(spread < 1e-4), (spread, mixed)
        # the fully mixed values are the printed ones (species mass over water
        # volume; on this coarse mesh within 0.5 % of 0.386 and 3 % of 0.023)
        assert abs(mixed[0] - 0.386) < 0.005 * 0.386 and abs(mixed[1] - 0.023) < 0.03 * 0.023, mixed
    else:
        assert np.all(spread > 0.1), spread


def test_uniform_concentration_stays_uniform_with_diffusion():
    sc = S.tiny_random(4, 4, seed=2, bcs=False)
    n = sc.n_cells
    sc = S.Scenario(**{**sc.__dict__, "phi0": np.full((1, n), 0.3),
                       "diffusion": S.Diffusion(Km=0.1, alpha_L=13.0, alpha_T=1.2, zeta=0.5)})
    sim = oracle.Sim(sc)
    sim.run_until(1.0)
    H, _, _, _ = sim.state()
    h = H - sim.bed()
    wet = h > 1e-3
    phi = sim.scalars()[0, wet] / h[wet]
    assert np.abs(phi - 0.3).max() <= 1e-12
    assert np.abs(sim.psi()).max() <= 1e-10


def test_dispersion_is_stronger_along_the_flow():
    # uniform flow (normal depth and discharge on a 1e-3 slope, Manning 0.03)
    # down a wide channel carries a Gaussian patch; with alpha_L = 13,
    # alpha_T = 1.2 the patch's variance grows faster along x than across it
    # (the ratio would be reversed with the coefficients swapped); the
    # molecular part is zero and the relaxation's own numerical diffusion,
    # isotropic, narrows the ratio
    S0, n_m, q = 1e-3, 0.03, 1.0
    hn = (n_m * q / np.sqrt(S0)) ** 0.6
    lx, ly, d = 120.0, 40.0, 1.0
    xy, tri, sides = M.structured_right(lx, ly, d)
    ncell = len(tri)
    segs = [M.segments_on_side(xy, sides["x0"], -1, 1e9, 1), M.segments_on_side(xy, sides["x1"], -1, 1e9, 1)]
    tags = [np.full(len(segs[0]), 1, np.int32), np.full(len(segs[1]), 2, np.int32)]
    c = xy[tri].mean(axis=1)
    phi0 = np.exp(-((c[:, 0] - 30.0) ** 2 + (c[:, 1] - 20.0) ** 2) / (2 * 3.0 ** 2))
    sc = S.Scenario("channel", np.c_[xy, S0 * (lx - xy[:, 0])], tri.astype(np.int32), np.concatenate(segs),
                    np.concatenate(tags),
                    [S.BC(1, S.INFLOW_UNIFORM, slope=S0, t=np.array([0.0]), Q=np.array([q * ly])),
                     S.BC(2, S.OUTFLOW_UNIFORM, slope=S0)], None, np.full(ncell, hn), np.full(ncell, q),
                    np.zeros(ncell), np.full(ncell, n_m), t_end=30.0, cfl=0.5, phi0=phi0[None, :],
                    diffusion=S.Diffusion(Km=0.0, alpha_L=13.0, alpha_T=1.2, zeta=2.0))
    sim = oracle.Sim(sc)
    area = sim.mesh.geometry()["area"]

    def moments():
        qs = sim.scalars()[0] * area
        m = qs.sum()
        mx, my = (qs * c[:, 0]).sum() / m, (qs * c[:, 1]).sum() / m
        return (qs * (c[:, 0] - mx) ** 2).sum() / m, (qs * (c[:, 1] - my) ** 2).sum() / m

    vx0, vy0 = moments()
    sim.run_until(30.0)
    vx, vy = moments()
    gx, gy = vx - vx0, vy - vy0
    print("variance growth along / across the flow", gx, gy, gx / gy)
    assert gy > 0 and gx > 3.0 * gy, (gx, gy)
