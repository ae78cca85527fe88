"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/bvc.h declares, and host-side validation returns error codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bvc.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bvc_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2302_11825_amd import _bvc

    lib = C.CDLL(_bvc.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert set(syms) <= set(_bvc.EXPORTED)


def test_scene_validation_errors():
    from paper_2302_11825_amd import _bvc

    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    seg = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.int32)
    h = _bvc.bvc_scene_create(2, sq, seg)
    info = _bvc.bvc_scene_get_info(h)
    assert info.n_prims == 4 and info.uploaded == 0 and info.device_bytes > 0
    assert abs(info.boundary_measure - 4.0) < 1e-15
    assert abs(info.diagonal - np.sqrt(2)) < 1e-15
    _bvc.bvc_scene_destroy(h)
    bad = sq.copy()
    bad[2, 0] = np.nan
    with pytest.raises(_bvc.BVCError) as e:
        _bvc.bvc_scene_create(2, bad, seg)
    assert e.value.code == -1
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_scene_create(2, sq, np.array([[0, 1], [1, 1]], np.int32))  # zero length
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_scene_create(2, sq, np.array([[0, 7]], np.int32))  # index out of range
    tri = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0.0]])
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_scene_create(3, tri, np.array([[0, 1, 2]], np.int32))  # zero area
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_scene_create(4, sq, seg)


def test_not_uploaded_scene_is_a_state_error():
    from paper_2302_11825_amd import _bvc

    h = _bvc.bvc_scene_create(2, wl.circle_polygon(16).verts, wl.circle_polygon(16).prims)
    rc = _bvc._L.bvc_classify(h, 10, None, 0.1, None, None, None)
    assert rc == -5
    _bvc.bvc_scene_destroy(h)


def test_candidate_measure_matches_oracle(orc):
    from paper_2302_11825_amd import _bvc

    for scene, sides in ((wl.circle_polygon(128), 1), (wl.star_polygon(1024, 3), 2),
                         (wl.displaced_icosphere(2, 5), 1)):
        h = _bvc.bvc_scene_create(scene.dim, scene.verts, scene.prims)
        m = _bvc.bvc_cache_measure(h, 0.01, sides)
        assert m == orc.Scene(scene).candidate_measure(0.01, sides)
        _bvc.bvc_scene_destroy(h)


def test_bvh_depth_bounds_stack():
    from paper_2302_11825_amd import _bvc

    for scene in (wl.star_polygon(4096), wl.displaced_icosphere(5, 1)):
        h = _bvc.bvc_scene_create(scene.dim, scene.verts, scene.prims)
        info = _bvc.bvc_scene_get_info(h)
        # surface-area splits down to level 32, median splits below it
        assert info.depth <= 32 + int(np.ceil(np.log2(scene.prims.shape[0] / 4)))
        assert info.depth >= int(np.ceil(np.log2(scene.prims.shape[0] / 4)))
        assert info.n_nodes >= scene.prims.shape[0] // 4 - 1  # internal nodes = leaves - 1
        _bvc.bvc_scene_destroy(h)


def test_argument_validation_without_gpu():
    from paper_2302_11825_amd import _bvc

    L = _bvc._L
    assert L.bvc_compact(-1, None, 1, None, None, C.byref(C.c_int64()), None) == -1
    assert L.bvc_take(7, 0, 1, None, 1, 1, None, 1, None, None) == -1
    assert L.bvc_gather_u(4, None, None, 1, None, None, None, None) == -1
    assert L.bvc_gather_multi(3, 1, None, None, 48, None, None, 1, None, None, 0, None, 0, None) == -4
    assert L.bvc_reduce_walks(1, 0, 0, None, None, None, None, None, 0, None, None, None) == -1
    assert L.bvc_cache_walks(None, None, 0, None, None, None, None, None, None, None, None, None, None,
                             None) == -1


def test_band_narrower_than_offset_is_rejected():
    from paper_2302_11825_amd import pipeline as pl

    prob = wl.problem_c1()
    with pytest.raises(ValueError, match="narrower than the offset"):
        pl.Prepared(prob, band=0.5 * prob.offset, device="cpu")
