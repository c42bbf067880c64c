"""Whole-step pins of the oracle against closed forms and the paper's printed
values: the wet-bed dam break (Stoker), the dry-bed dam break (Ritter), the
two-rarefaction problem of T5 and the resting level of T6."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import swe_inputs as S
from exact_riemann import RiemannSWE

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def column_average(sc, H, d, length=100.0):
    """Average depth of each d-wide column of the structured channel (all
    cells of a column have the same area)."""
    cx = sc.centroids()[:, 0]
    k = np.floor(cx / d).astype(int)
    n = int(round(length / d))
    return np.bincount(k, H, n) / np.bincount(k, None, n)


def run_channel(sc, d, t_end):
    sim = oracle.Sim(sc)
    sim.run_until(t_end)
    H, qx, qy, t = sim.state()
    assert t == t_end
    return sim, column_average(sc, H, d), column_average(sc, qx, d)


def test_stoker_wet_bed_dam_break_converges():
    ex = RiemannSWE(1.0, 0.0, 0.1, 0.0)
    assert abs(ex.hs - 0.396175) < 1e-6
    errs = []
    for d in (1.0, 0.5, 0.25):
        sc = S.dam_break(d, h_right=0.1)
        sim, h, _ = run_channel(sc, d, 5.0)
        xl = np.arange(len(h)) * d
        he = ex.cell_average(xl, xl + d, 5.0, 50.0, sub=16)
        errs.append(np.abs(h - he).sum() * d / 100.0)
        xc = xl + 0.5 * d
        plateau = h[(xc > 53.0) & (xc < 63.0)].mean()
        assert abs(plateau - ex.hs) / ex.hs < 0.01
        dg = sim.diag()
        assert dg["clipped"] == 0.0
        assert abs(dg["mass"] - 550.0) < 1e-11 * 550.0
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.004


def test_ritter_dry_bed_dam_break():
    ex = RiemannSWE(1.0, 0.0, 0.0, 0.0)
    front_exact = 50.0 + 2.0 * ex.cL * 5.0
    assert abs(front_exact - 81.32) < 0.01
    errs, lags = [], []
    for d in (1.0, 0.5, 0.25):
        sc = S.dam_break(d, h_right=0.0)
        sim, h, _ = run_channel(sc, d, 5.0)
        xl = np.arange(len(h)) * d
        he = ex.cell_average(xl, xl + d, 5.0, 50.0, sub=16)
        errs.append(np.abs(h - he).sum() * d / 100.0)
        front = (xl + 0.5 * d)[h > 1e-3].max()
        lags.append(front_exact - front)
        dg = sim.diag()
        # conservative up to the volume the positivity clip adds
        assert abs(dg["mass"] - dg["clipped"] - 500.0) < 1e-11 * 500.0
        assert dg["clipped"] < 1e-4 * 500.0
    assert errs[0] > errs[1] > errs[2]
    assert lags[0] > lags[1] > lags[2] >= 0.0
    assert lags[2] < 1.5


def test_t5_two_rarefactions():
    g = GOLD["t5_setup"]
    ex = RiemannSWE(g["h"], g["qx_left"] / g["h"], g["h"], g["qx_right"] / g["h"])
    assert abs(ex.hs - 0.271532) < 1e-6 and abs(ex.us) < 1e-14
    errs = []
    for d, tol in ((0.1, 3e-3), (0.05, 6e-4)):
        sc = S.t5_rarefactions(d, t_end=g["t_end"])
        assert sc.cfl == g["cfl"]
        sim, h, q = run_channel(sc, d, g["t_end"])
        xl = np.arange(len(h)) * d
        he = ex.cell_average(xl, xl + d, g["t_end"], g["x_split"], sub=8)
        errs.append(np.abs(h - he).sum() * d / 100.0)
        mid = len(h) // 2
        assert np.all(np.abs(h[mid - 2:mid + 2] - ex.hs) < tol)
        # the star region between the two rarefaction tails is at rest
        xc = xl + 0.5 * d
        star = np.abs(xc - g["x_split"]) < 3.0
        assert np.abs(q[star]).max() < 0.02
    assert errs[1] < errs[0] < 2e-3


def test_t6_relaxes_to_the_printed_rest_depth():
    sc = S.t6_three_humps(n_cells=5000, t_end=1200.0)
    sim = oracle.Sim(sc)
    geo = sim.mesh.geometry()
    area, zb = geo["area"], geo["zb"]
    H0 = sim.state()[0]
    V0 = ((H0 - zb) * area).sum()
    # discrete level at which the same volume lies flat over this bed
    H_rest = brentq(lambda L: (np.maximum(0.0, L - zb) * area).sum() - V0, 0.0, 3.0, xtol=1e-14)
    gold = GOLD["t6_rest_depth"]
    assert abs(H_rest - gold["value"]) <= 0.5 * 10 ** -gold["printed_decimals"] + 1e-3
    m0 = sim.diag()["mass"]
    sim.run_until(1200.0)
    H, qx, qy, _ = sim.state()
    wet = (H - zb) > 1e-2
    assert np.all(np.abs(H[wet] - H_rest) < 1e-3)
    dg = sim.diag()
    assert dg["clipped"] == 0.0
    assert abs(dg["mass"] - m0) < 1e-12 * m0


def test_t6_reading_of_the_initial_condition():
    # continuous volume balance: reading the 0.125 m of the initial condition
    # as a surface elevation reproduces the printed rest depth; reading it as
    # a depth does not
    x = np.linspace(0, 75, 1501)
    y = np.linspace(-15, 15, 601)
    X, Y = np.meshgrid(0.5 * (x[1:] + x[:-1]), 0.5 * (y[1:] + y[:-1]))
    eta = S.configs.t6_bed(X, Y)
    dA = (x[1] - x[0]) * (y[1] - y[0])
    level = lambda V: brentq(lambda L: np.maximum(0, L - eta).sum() * dA - V, 0, 4)  # noqa: E731
    v_surface = np.maximum(0, np.where(X < 16, 1.0, 0.125) - eta).sum() * dA
    v_depth = (np.where(X < 16, 1.0, 0.125) * np.ones_like(eta)).sum() * dA
    assert abs(level(v_surface) - 0.364) < 1e-3
    assert abs(level(v_depth) - 0.364) > 0.02
