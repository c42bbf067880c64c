"""CPU checks of the HIP library that need no GPU: it loads, exports every
function include/swe.h declares, and its host mesh preparation (edge
matching, boundary tags, validation) agrees with the oracle's own."""
import os
import re

import numpy as np
import pytest

import oracle
import swe_inputs as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe.h")


@pytest.fixture(scope="module")
def swe():
    from paper_2102_12862_amd import swe as mod
    mod.load()
    return mod


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(swe_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ("swe_mesh_create", "swe_state_init", "swe_step", "swe_run_until", "swe_state_read", "swe_mass"):
        assert n in names


def test_library_exports_every_declared_symbol(swe):
    import ctypes
    lib = ctypes.CDLL(swe.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers exactly the declared functions
    assert sorted(swe.SIGNATURES) == declared_functions()


def test_params_defaults(swe):
    p = swe.params()
    assert p.g == 9.81 and p.cfl == 0.9 and p.h_min == 1e-4 and np.isinf(p.dt_max)
    assert p.precision == swe.FP64 and p.renumber == 1 and p.friction == swe.FRICTION["manning"]
    assert p.limiter == swe.LIMIT_NONE


@pytest.mark.parametrize("maker", [lambda: S.lake_at_rest(3000), lambda: S.valley_flood(20000, scale=0.1),
                                   lambda: S.tiny_random(3, 3, seed=1), lambda: S.dam_break(1.0)])
def test_mesh_counts_match_the_oracle(swe, maker):
    sc = maker()
    for renumber in (True, False):
        m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=False, renumber=renumber)
        info = m.info()
        om = oracle.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag)
        assert info["n_cells"] == sc.n_cells
        assert info["n_edges"] == om.n_edges
        assert info["n_boundary_edges"] == om.n_boundary_edges
        assert m.footprint(swe.FP32) > 40 * sc.n_cells


def test_mesh_validation(swe):
    sc = S.tiny_random(2, 2, seed=0)
    bad = sc.nodes.copy()
    bad[sc.tri[0, 1]] = bad[sc.tri[0, 0]]
    cases = [
        (bad, sc.tri, None, None, "degenerate"),
        (sc.nodes, np.vstack([sc.tri, sc.tri[:1]]), None, None, ("non-conforming", "orientation")),
        (sc.nodes, sc.tri, np.array([[0, len(sc.nodes) - 1]], np.int32), np.array([1], np.int32), "not an edge of the mesh"),
        (np.where(np.arange(sc.nodes.size).reshape(sc.nodes.shape) == 4, np.nan, sc.nodes), sc.tri, None, None,
         "non-finite"),
        (sc.nodes, np.where(sc.tri == sc.tri[0, 0], len(sc.nodes) + 5, sc.tri).astype(np.int32), None, None,
         "vertex index"),
    ]
    for nodes, tri, seg, tag, what in cases:
        with pytest.raises(swe.SweError) as e:
            swe.Mesh(nodes, tri, seg, tag, device=False)
        assert e.value.code == swe.EINVAL
        assert any(w in str(e.value) for w in ((what,) if isinstance(what, str) else what))


def test_clockwise_input_is_accepted(swe):
    sc = S.tiny_random(3, 3, seed=2)
    t = sc.tri.copy()
    t[:, 1], t[:, 2] = sc.tri[:, 2], sc.tri[:, 1]
    m = swe.Mesh(sc.nodes, t, sc.bnd_seg, sc.bnd_tag, device=False)
    assert m.info()["n_edges"] == oracle.Mesh(sc.nodes, sc.tri).n_edges


@pytest.mark.parametrize("maker", [lambda: S.lake_at_rest(3000), lambda: S.valley_flood(20000, scale=0.1),
                                   lambda: S.tiny_random(3, 3, seed=1), lambda: S.tiny_random(1, 1, seed=4),
                                   lambda: S.dam_break(1.0)])
def test_tile_edge_lists_cover_every_cell_edge_once(swe, maker):
    sc = maker()
    for renumber in (True, False):
        m = swe.Mesh(sc.nodes, sc.tri, sc.bnd_seg, sc.bnd_tag, device=False, renumber=renumber)
        for tile in (128, 256, 512):
            m.check(tile)
    with pytest.raises(swe.SweError):
        m.check(100)
