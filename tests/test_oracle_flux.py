"""Pins of the oracle's single-edge pieces: the HLLC flux and the friction
split, against properties the mathematics fixes (not against a retyped
formula)."""
import math

import numpy as np
import pytest

import oracle

G = 9.81


def phys(h, un, ut):
    return np.array([h * un, h * un * un + 0.5 * G * h * h, h * un * ut])


def hll_mass(hL, uL, hR, uR, SL, SR):
    FL, FR = hL * uL, hR * uR
    return (SR * FL - SL * FR + SL * SR * (hR - hL)) / (SR - SL)


def speeds(hL, uL, hR, uR):
    cL, cR = math.sqrt(G * hL), math.sqrt(G * hR)
    a = 0.5 * (cL + cR) + 0.25 * (uL - uR)
    us = 0.5 * (uL + uR) + cL - cR
    cs = max(0.0, a)
    return min(uL - cL, us - cs), max(uR + cR, us + cs)


def test_consistency_identical_states_bitwise():
    rng = np.random.default_rng(1)
    for _ in range(200):
        h, un, ut = rng.uniform(0.01, 3), rng.uniform(-4, 4), rng.uniform(-4, 4)
        F = oracle.hllc(h, un, ut, h, un, ut)
        assert np.array_equal(F, phys(h, un, ut))


def test_consistency_is_continuous():
    # a state a hair away from identical gives the physical flux to O(eps)
    rng = np.random.default_rng(2)
    for _ in range(200):
        h, un, ut = rng.uniform(0.1, 3), rng.uniform(-4, 4), rng.uniform(-4, 4)
        F = oracle.hllc(h, un, ut, h * (1 + 1e-12), un, ut)
        assert np.allclose(F, phys(h, un, ut), rtol=1e-9, atol=1e-9)


def test_dry_dry_is_zero():
    assert np.array_equal(oracle.hllc(0.0, 1.0, 2.0, 0.0, -1.0, 3.0), np.zeros(3))


def test_supersonic_upwinding():
    # all waves move right (u - c >= 0): the flux is the left physical flux
    for hL, uL, hR, uR in [(1.0, 5.0, 0.8, 5.5), (0.5, 3.0, 0.5, 3.2), (2.0, 6.0, 0.0, 0.0)]:
        F = oracle.hllc(hL, uL, 0.7, hR, uR, -0.2)
        assert np.array_equal(F, phys(hL, uL, 0.7))
    # all waves move left: the right physical flux
    F = oracle.hllc(0.9, -6.0, 0.1, 1.0, -5.5, 0.4)
    assert np.array_equal(F, phys(1.0, -5.5, 0.4))


def test_mass_flux_equals_hll():
    # The HLLC middle states carry the HLL-average depth on both sides of the
    # contact, so the HLLC mass flux equals the HLL mass flux for the same
    # wave speeds.  A wrong sign, index or transposed operand in the contact
    # speed S* or in the star states breaks this.
    rng = np.random.default_rng(3)
    for _ in range(500):
        hL, hR = rng.uniform(0.05, 3, 2)
        uL, uR, vL, vR = rng.uniform(-3, 3, 4)
        SL, SR = speeds(hL, uL, hR, uR)
        F = oracle.hllc(hL, uL, vL, hR, uR, vR)
        if SL >= 0:
            ref = hL * uL
        elif SR <= 0:
            ref = hR * uR
        else:
            ref = hll_mass(hL, uL, hR, uR, SL, SR)
        assert abs(F[0] - ref) <= 1e-12 * (1 + abs(ref))


def test_isolated_shear_wave_is_exact():
    # equal depth and normal velocity, different tangential velocity: an
    # isolated contact; HLLC resolves it exactly (HLL would smear it)
    for un in (0.7, -0.7):
        F = oracle.hllc(1.3, un, 2.0, 1.3, un, -1.0)
        up = 2.0 if un > 0 else -1.0
        assert np.allclose(F, phys(1.3, un, up), rtol=1e-13, atol=1e-13)


def test_tangential_flux_is_mass_flux_times_upwind_tangential_velocity():
    rng = np.random.default_rng(4)
    for _ in range(300):
        hL, hR = rng.uniform(0.05, 3, 2)
        uL, uR, vL, vR = rng.uniform(-3, 3, 4)
        F = oracle.hllc(hL, uL, vL, hR, uR, vR)
        assert min(abs(F[2] - F[0] * vL), abs(F[2] - F[0] * vR)) <= 1e-12 * (1 + abs(F[2]))


def test_reflection_symmetry():
    # swapping the sides and reversing the normal negates mass and tangential
    # fluxes and keeps the normal-momentum flux (up to rounding)
    rng = np.random.default_rng(5)
    for _ in range(300):
        hL, hR = rng.uniform(0.0, 3, 2) * (rng.random(2) > 0.15)
        uL, uR, vL, vR = rng.uniform(-3, 3, 4)
        F = oracle.hllc(hL, uL, vL, hR, uR, vR)
        Fm = oracle.hllc(hR, -uR, vR, hL, -uL, vL)
        s = 1e-12 * (1 + np.abs(F).max())
        assert abs(F[0] + Fm[0]) <= s and abs(F[1] - Fm[1]) <= s and abs(F[2] + Fm[2]) <= s


def test_dry_bed_front_speeds():
    # water on the left of a dry bed: the Ritter front moves at u + 2c; the
    # fastest HLLC wave is that front, so with the left wave fully
    # supersonic the flux is the left flux, and otherwise the mass flux is
    # the HLL one built on (u - c, u + 2c)
    hL, uL = 1.0, 0.5
    c = math.sqrt(G * hL)
    F = oracle.hllc(hL, uL, 0.0, 0.0, 0.0, 0.0)
    SL, SR = uL - c, uL + 2 * c
    ref = (SR * hL * uL + SL * SR * (0 - hL)) / (SR - SL)
    assert abs(F[0] - ref) <= 1e-13
    # mirror: dry on the left
    Fm = oracle.hllc(0.0, 0.0, 0.0, hL, -uL, 0.0)
    assert abs(Fm[0] + ref) <= 1e-13


def _rk4_friction(q0, h, gn2, dt, n=20000):
    # dq/dt = -g n^2 |q| q / h^(7/3), integrated with many small RK4 steps
    kappa = gn2 / h ** (7.0 / 3.0)
    f = lambda q: -kappa * np.linalg.norm(q) * q  # noqa: E731
    q = np.array(q0, float)
    k = dt / n
    for _ in range(n):
        a = f(q); b = f(q + 0.5 * k * a); c = f(q + 0.5 * k * b); d = f(q + k * c)
        q = q + k / 6.0 * (a + 2 * b + 2 * c + d)
    return q


@pytest.mark.parametrize("q0,h,n,dt", [((1.0, 0.5), 0.8, 0.035, 0.5), ((-3.0, 2.0), 0.3, 0.06, 2.0),
                                       ((0.2, -0.1), 2.0, 0.025, 10.0)])
def test_friction_split_solves_the_ode(q0, h, n, dt):
    gn2 = G * n * n
    f = oracle.friction_factor(math.hypot(*q0), h, gn2, dt)
    q_or = f * np.array(q0)
    q_rk = _rk4_friction(q0, h, gn2, dt)
    assert np.allclose(q_or, q_rk, rtol=1e-9, atol=1e-12)


def test_friction_thin_film_and_frictionless():
    assert oracle.friction_factor(1.0, 5e-5, 0.01, 1.0) == 0.0
    assert oracle.friction_factor(1.0, 0.5, 0.0, 1.0) == 1.0
