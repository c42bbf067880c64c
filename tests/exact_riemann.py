"""Exact solution of the 1D shallow-water Riemann problem on a flat bed.

Independent closed form used to pin the oracle (Toro 2001, the textbook the
paper cites for the SWE and for HLLC): the star depth solves
f_L(h) + f_R(h) + (u_R - u_L) = 0 with rarefaction branches
2(sqrt(g h) - sqrt(g h_K)) and shock branches
(h - h_K) sqrt(g (h + h_K) / (2 h h_K)); dry-bed and dry-middle cases use the
Riemann invariants u + 2c and u - 2c.  Written from the mathematics, with a
bracketing root finder, and sharing nothing with the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

G = 9.81


def _f(h, hk, g):
    if h <= hk:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
    return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))


class RiemannSWE:
    def __init__(self, hL, uL, hR, uR, g=G):
        self.hL, self.uL, self.hR, self.uR, self.g = hL, uL, hR, uR, g
        cL = math.sqrt(g * hL)
        cR = math.sqrt(g * hR)
        self.cL, self.cR = cL, cR
        if hL > 0 and hR > 0 and 2.0 * (cL + cR) > uR - uL:
            self.kind = "wet"
            fun = lambda h: _f(h, hL, g) + _f(h, hR, g) + uR - uL  # noqa: E731
            hi = max(hL, hR)
            while fun(hi) < 0:
                hi *= 2.0
            self.hs = brentq(fun, 1e-14, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
            self.us = 0.5 * (uL + uR) + 0.5 * (_f(self.hs, hR, g) - _f(self.hs, hL, g))
            self.cs = math.sqrt(g * self.hs)
        elif hL > 0 and hR <= 0:
            self.kind = "dry_right"
        elif hL <= 0 and hR > 0:
            self.kind = "dry_left"
        else:
            self.kind = "dry_middle"

    # -- sampling -----------------------------------------------------------
    def _left_fan(self, S):
        c = (self.uL + 2 * self.cL - S) / 3.0
        return c * c / self.g, (self.uL + 2 * self.cL + 2 * S) / 3.0

    def _right_fan(self, S):
        c = (-self.uR + 2 * self.cR + S) / 3.0
        return c * c / self.g, (self.uR - 2 * self.cR + 2 * S) / 3.0

    def sample(self, S: float):
        """(h, u) at similarity coordinate S = x/t."""
        hL, uL, hR, uR, g = self.hL, self.uL, self.hR, self.uR, self.g
        cL, cR = self.cL, self.cR
        if self.kind == "wet":
            hs, us, cs = self.hs, self.us, self.cs
            if S <= us:
                if hs > hL:  # left shock
                    sl = uL - cL * math.sqrt(0.5 * (hs + hL) * hs) / hL
                    return (hL, uL) if S <= sl else (hs, us)
                head, tail = uL - cL, us - cs
                if S <= head:
                    return hL, uL
                if S >= tail:
                    return hs, us
                return self._left_fan(S)
            if hs > hR:  # right shock
                sr = uR + cR * math.sqrt(0.5 * (hs + hR) * hs) / hR
                return (hR, uR) if S >= sr else (hs, us)
            head, tail = uR + cR, us + cs
            if S >= head:
                return hR, uR
            if S <= tail:
                return hs, us
            return self._right_fan(S)
        if self.kind == "dry_right":
            if S <= uL - cL:
                return hL, uL
            if S >= uL + 2 * cL:
                return 0.0, 0.0
            return self._left_fan(S)
        if self.kind == "dry_left":
            if S >= uR + cR:
                return hR, uR
            if S <= uR - 2 * cR:
                return 0.0, 0.0
            return self._right_fan(S)
        # two rarefactions separated by a dry region
        if S <= uL - cL:
            return hL, uL
        if S <= uL + 2 * cL:
            return self._left_fan(S)
        if S >= uR + cR:
            return hR, uR
        if S >= uR - 2 * cR:
            return self._right_fan(S)
        return 0.0, 0.0

    def profile(self, x: np.ndarray, t: float, x0: float):
        hu = np.array([self.sample((xi - x0) / t) for xi in x])
        return hu[:, 0], hu[:, 1]

    def cell_average(self, x_lo, x_hi, t, x0, sub=64):
        """Exact solution averaged over [x_lo, x_hi] (midpoint rule on sub cells)."""
        out = np.zeros(len(x_lo))
        for i, (a, b) in enumerate(zip(x_lo, x_hi)):
            xs = a + (np.arange(sub) + 0.5) * (b - a) / sub
            out[i] = np.mean([self.sample((x - x0) / t)[0] for x in xs])
        return out
