"""The FP32 state's water surface: an FP32 high part plus a 16-bit low part
in units of 2^-16 of an ulp of the high part, so that the surface resolves
to about 2^-40 of itself.  A state reads its initial surface back to within
2^-39 of itself over nine decades and both signs (an FP32 surface alone:
2^-25), and increments far below half an ulp of the FP32 surface are kept
step after step: rain of 1 mm/h on water standing at 100 m elevation adds
about 3e-8 m per step (dt about 0.1 s) against an FP32 spacing of 7.6e-6 m
there, all of which an FP32 surface alone would round away."""
import numpy as np
import pytest

import swe_inputs as S
from swe_inputs import mesh as M
from gpu_util import gpu_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swe():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import swe as mod
    return mod


def _flat(H0, z, **kw):
    xy, tri, _ = M.structured_right(20.0, 10.0, 1.0)
    n = len(tri)
    return S.Scenario("flat", np.c_[xy, np.full(len(xy), z)], tri.astype(np.int32), np.zeros((0, 2), np.int32),
                      np.zeros(0, np.int32), [], np.broadcast_to(H0, (n,)).copy(), None, np.zeros(n), np.zeros(n),
                      np.full(n, 0.02), t_end=60.0, dt_max=0.5, cfl=0.5, **kw)


def test_surface_reads_back_to_2e39(swe):
    n = len(M.structured_right(20.0, 10.0, 1.0)[1])
    r = np.random.default_rng(11)
    H0 = np.where(r.random(n) < 0.5, -1.0, 1.0) * 10.0 ** r.uniform(-3.0, 6.0, n)
    st = gpu_state(_flat(H0, -2e6), swe.FP32)
    H = st.read()["H"]
    rel = np.abs(H - H0) / np.abs(H0)
    assert rel.max() <= 2.0 ** -39, rel.max()
    # an FP32 surface alone could not do this
    f32 = np.abs(H0.astype(np.float32).astype(np.float64) - H0) / np.abs(H0)
    assert f32.max() > 2.0 ** -30


def test_rain_far_below_the_fp32_spacing_is_kept(swe):
    n = len(M.structured_right(20.0, 10.0, 1.0)[1])
    rain = S.Source(S.SRC_EXACT, S.SRC_INTENSITY, np.array([0.0]), np.array([1.0]))  # 1 mm/h
    sc = _flat(100.0, 99.5, sources=(rain,), src_region=np.zeros(n, np.int32))
    st = gpu_state(sc, swe.FP32)
    steps = st.run_until(50.0)
    r = st.read()
    assert np.all(r["qx"] == 0.0) and np.all(r["qy"] == 0.0) and np.ptp(r["H"]) == 0.0
    gain = 1.0 / 3.6e6 * 50.0
    assert gain / steps < 0.01 * float(np.spacing(np.float32(100.0)))
    # each step rounds the surface to the low part's unit 2^(7-40) at 100 m
    unit = 2.0 ** (7 - 40)
    assert np.max(np.abs(r["h"] - (0.5 + gain))) <= steps * unit / 2 + 1e-15
    assert abs(st.mass()["mass"] - 200.0 * (0.5 + gain)) <= 200.0 * steps * unit
    assert abs(st.source_volume() - 200.0 * gain) <= 1e-12 * 200.0
