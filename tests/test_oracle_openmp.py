"""The OpenMP build of the oracle (the same C source with its edge and cell
loops spread over the host's cores) against the serial build: every
result bitwise equal, including the boundary-flux integral, the clipped
volume and the source volume, whose sums it keeps in the serial order.  Its
timing is the all-core CPU baseline; its results stand for the serial
oracle's on the workloads too large to step serially in a test."""
import numpy as np
import pytest

import oracle
import swe_inputs as S


def _same(a, b, steps):
    a.run_steps(steps)
    b.run_steps(steps)
    A, B = a.state(), b.state()
    for x, y in zip(A[:3], B[:3]):
        assert np.array_equal(x, y)
    assert A[3] == B[3]
    assert a.diag() == b.diag()


@pytest.mark.parametrize("which", ["tiny", "ritter", "valley_dry", "valley_wet"])
def test_openmp_build_is_bitwise_the_serial_one(which):
    oracle.threads(4)
    s = float(np.sqrt(30000 / 4e6))
    sc = {"tiny": lambda: S.tiny_random(5, 4, seed=7),
          "ritter": lambda: S.dam_break(1.0, h_right=0.0),
          "valley_dry": lambda: S.valley_flood(n_cells=30000, scale=s),
          "valley_wet": lambda: S.valley_flood(n_cells=30000, scale=s, snapshot="wet")}[which]()
    _same(oracle.Sim(sc), oracle.Sim(sc, omp=True), 60)


def test_openmp_build_with_sources_clips_and_walls():
    # a sink that takes what the cells hold (source tally) under a dam break
    # over a dry bed (clips), then an exact sink that runs dry (an error)
    sc = S.dam_break(1.0, h_right=0.0)
    n = sc.n_cells
    cx = sc.centroids()[:, 0]
    region = np.where(cx > 70.0, 0, -1).astype(np.int32)
    for mode in (S.SRC_AVAILABLE, S.SRC_EXACT):
        src = S.Source(mode, S.SRC_DISCHARGE, np.array([0.0]), np.array([-5.0]))
        s2 = S.Scenario(**{**sc.__dict__, "sources": (src,), "src_region": region})
        a, b = oracle.Sim(s2), oracle.Sim(s2, omp=True)
        if mode == S.SRC_AVAILABLE:
            _same(a, b, 400)
            assert a.diag()["clipped"] > 0.0 and a.source_volume() < 0.0
        else:
            with pytest.raises(oracle.OracleError):
                a.run_steps(400)
            with pytest.raises(oracle.OracleError):
                b.run_steps(400)
            A, B = a.state(), b.state()
            for x, y in zip(A[:3], B[:3]):
                assert np.array_equal(x, y)
        assert a.diag() == b.diag() and a.source_volume() == b.source_volume()


def test_set_bed_keeps_the_surface_or_the_depth():
    sc = S.tiny_random(3, 3, seed=2)
    sim = oracle.Sim(sc)
    H0, qx0, qy0, _ = sim.state()
    z0 = sim.bed()
    z1 = z0 + 0.01
    sim.set_bed(z1)                       # depth kept
    H1, _, _, _ = sim.state()
    assert np.array_equal(sim.bed(), z1)
    assert np.allclose(H1 - z1, H0 - z0, rtol=0, atol=1e-15)
    sim.set_bed(z0, H0)                   # surface given
    assert np.array_equal(sim.state()[0], np.maximum(H0, z0))
    with pytest.raises(oracle.OracleError):
        sim.set_bed(np.full(sc.n_cells, np.nan))
