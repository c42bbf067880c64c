"""Linear stability of the step as read (eq. CFL_condition with rho = twice
the centroid-edge distance): a lake at rest perturbed by 1e-6 m must not
grow.  Holds at the default CFL 0.9 on the quality Delaunay meshes the
workloads use (every angle above 28 degrees, bumpy bed with dry islands), and
at CFL 0.5 on structured right triangles; on right triangles CFL 0.9 lets the
perturbation grow to order one, which is why the right-triangle generators of
long runs use 0.5 (the short dam-break runs keep 0.9)."""
import numpy as np
import pytest

import oracle
import swe_inputs as S
from swe_inputs import mesh as M


def _growth(sc, level, steps=120):
    rng = np.random.default_rng(0)
    H0 = level + 1e-6 * rng.standard_normal(sc.n_cells)
    sim = oracle.Sim(S.Scenario(**{**sc.__dict__, "H0": H0, "h0": None}))
    zb = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag).geometry()["zb"]
    wet = (level - zb) > 0.05
    try:
        for _ in range(steps):
            sim.step()
    except oracle.OracleError:
        return np.inf
    H = sim.state()[0]
    return float(np.abs(H[wet] - level).max())


def _right_triangles(cfl):
    xy, tri, _ = M.structured_right(40.0, 20.0, 1.0)
    n = len(tri)
    return S.Scenario("flat_right", np.c_[xy, np.zeros(len(xy))], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                      np.zeros(0, np.int32), [], None, np.full(n, 0.6), np.zeros(n), np.zeros(n), np.zeros(n),
                      t_end=1e9, cfl=cfl)


def test_delaunay_lake_stable_at_default_cfl():
    assert _growth(S.lake_at_rest(3000), 1.5) < 1e-5


def test_right_triangles_stable_at_half_cfl():
    assert _growth(_right_triangles(0.5), 0.6) < 1e-5


def test_right_triangles_grow_at_default_cfl():
    # documents the limit of the printed time step on this mesh type
    assert _growth(_right_triangles(0.9), 0.6) > 1e-2
