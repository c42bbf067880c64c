"""Serving: requests arriving while others run are admitted as footprint
frees up, share the device through one persistent kernel per step, and each
result equals the same request solved alone, bit for bit."""
import numpy as np
import pytest

import swe_inputs as S
from gpu_util import device, gpu_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def modules():
    import torch
    assert torch.cuda.is_available()
    from paper_2102_12862_amd import serve, swe
    return serve, swe


def _requests(serve):
    arrive, sizes, horizon = S.serving_trace(n_requests=6, rate=20.0, n_lo=4000, n_hi=30000, h_lo=20.0, h_hi=60.0)
    scen = {i: S.serving_request(i, int(n), float(h)) for i, (n, h) in enumerate(zip(sizes, horizon))}
    return [serve.Request(i, float(a), (lambda sc=scen[i]: sc), float(horizon[i])) for i, a in enumerate(arrive)], scen


def test_served_results_equal_solo_runs(modules):
    serve, swe = modules
    reqs, scen = _requests(serve)
    sizes = sorted(sc.n_cells for sc in scen.values())
    # room for about three of the requests at a time, so admission binds
    mesh = swe.Mesh(scen[0].nodes, scen[0].tri, scen[0].bnd_seg, scen[0].bnd_tag, device=device())
    per_cell = mesh.footprint(swe.FP32) / scen[0].n_cells
    budget = int(per_cell * (sizes[-1] + sizes[-2] + sizes[-3]) * 1.05)
    srv = serve.Server(precision=swe.FP32, budget_bytes=budget, steps_per_round=16, device=device())
    srv.serve(reqs)
    srv.close()
    for r in reqs:
        assert r.error is None, r.error
        assert r.result["t"] == r.t_end
        st = gpu_state(scen[r.rid], swe.FP32)
        st.run_until(r.t_end)
        solo = st.read()
        for f in ("H", "qx", "qy"):
            assert np.array_equal(r.result[f], solo[f]), (r.rid, f)
    summ = serve.summarize(reqs, wall=max(r.finished for r in reqs))
    assert summ["errors"] == 0 and summ["p99_s"] >= summ["p50_s"] > 0
    print(summ)


def test_sequential_baseline_matches(modules):
    serve, swe = modules
    reqs, scen = _requests(serve)
    reqs = reqs[:3]
    serve.serve_sequential(reqs, precision=swe.FP32, device=device())
    for r in reqs:
        st = gpu_state(scen[r.rid], swe.FP32)
        st.run_until(r.t_end)
        assert np.array_equal(r.result["H"], st.read()["H"])
