"""Autotuned launch shapes (marked gpu): the tuners pick among shapes that
compute the same results, so every tuned launch must reproduce the default
launch bit for bit, for the gather (points per thread) and for the walks
(persistent grid size, traversal-loop exit threshold, and in 3D whether the
slab bounds prune the traversal)."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import c2_like_fields, lib, small_star

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dim", [2, 3])
def test_tuned_gather_is_bit_identical(dim):
    _bvc, pl = lib()
    say(f"tune gather dim={dim}")
    rng = np.random.default_rng(60 + dim)
    N, K, M = 3000, 70001, 900
    d = rng.normal(0, 1, (N, dim))
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", torch.float32)
    cy = d / np.linalg.norm(d, axis=1, keepdims=True)
    cache = dict(n=N, dtype=_bvc.F32, x=dev(cy), nrm=dev(cy), a=dev(rng.normal(0, 1, N) / N),
                 b=dev(rng.normal(0, 1, N) / N))
    src = dict(n=M, dtype=_bvc.F32, y=dev(rng.uniform(-0.5, 0.5, (M, dim))), s=dev(rng.normal(0, 1, M) / M))
    x = dev(rng.uniform(-0.8, 0.8, (K, dim)))
    u0 = torch.empty(K, dtype=torch.float32, device="cuda")
    g0 = torch.empty(dim, K, dtype=torch.float32, device="cuda")
    _bvc.bvc_gather_grad(dim, cache, src, K, x, u0, g0)
    u1, g1 = torch.empty_like(u0), torch.empty_like(g0)
    ppt = _bvc.bvc_tune_gather(dim, cache, src, K, x, u1, g1, reps=2)
    u2, g2 = torch.empty_like(u0), torch.empty_like(g0)
    _bvc.bvc_gather_grad(dim, cache, src, K, x, u2, g2)
    torch.cuda.synchronize()
    say(f"  chosen points per thread: {ppt}")
    assert ppt in (1, 2, 4)
    for u, g in ((u1, g1), (u2, g2)):
        assert torch.equal(u, u0) and torch.equal(g, g0)


def test_tuned_walks_are_bit_identical():
    _bvc, pl = lib()
    say("tune walks")
    g, f = c2_like_fields()
    sc = pl.Scene(small_star())
    gd, fd = pl.DeviceField(g), pl.DeviceField(f)
    cache = pl.sample_cache(sc, 4000, 1.5e-2, 2, 5, 0)
    params = pl.walk_params(3e-3, 32, 77, gd, fd, "f32")
    U0, D0, rec0, c0 = pl.cache_walks(sc, cache, params, "f32")
    n, W = cache.n, 32
    U1, D1 = torch.empty_like(U0), torch.empty_like(D0)
    ex, w1 = torch.empty_like(rec0["exit"]), torch.empty_like(rec0["w1"])
    c1 = torch.zeros(4, dtype=torch.int64, device="cuda")
    bpc, lanes, slabs = _bvc.bvc_tune_walks(sc.h, params, n, cache.x, cache.nrm, cache.R0, cache.xbar, U1, D1, ex, w1,
                                            c1, reps=1)
    U2, D2, rec2, c2 = pl.cache_walks(sc, cache, params, "f32")
    torch.cuda.synchronize()
    say(f"  chosen blocks per CU {bpc}, open lanes {lanes}")
    assert bpc in (4, 8, 16) and lanes in (0, 8, 16, 32, 48) and slabs == 0
    k = n * W
    for U, D in ((U1, D1), (U2, D2)):
        assert torch.equal(U[:k], U0[:k]) and torch.equal(D[:k], D0[:k])
    assert torch.equal(rec2["exit"][:, :k], rec0["exit"][:, :k])
    assert torch.equal(c2[1:], c0[1:]) and torch.equal(c1[1:], c0[1:])


def test_tuned_walks_3d_are_bit_identical():
    _bvc, pl = lib()
    say("tune walks 3D")
    scene = wl.displaced_icosphere(3, 31)
    g = wl.solid_harmonics_3d(np.random.default_rng(1).normal(0, 1, 16), 3)
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    cache = pl.sample_cache(sc, 6000, 2e-2, 1, 5, 0)
    params = pl.walk_params(4e-3, 16, 78, gd, None, "f32")
    U0, D0, rec0, c0 = pl.cache_walks(sc, cache, params, "f32")
    n, W = cache.n, 16
    U1, D1 = torch.empty_like(U0), torch.empty_like(D0)
    ex, w1 = torch.empty_like(rec0["exit"]), torch.empty_like(rec0["w1"])
    c1 = torch.zeros(4, dtype=torch.int64, device="cuda")
    bpc, lanes, slabs = _bvc.bvc_tune_walks(sc.h, params, n, cache.x, cache.nrm, cache.R0, cache.xbar, U1, D1, ex, w1,
                                            c1, reps=1)
    U2, D2, rec2, c2 = pl.cache_walks(sc, cache, params, "f32")
    torch.cuda.synchronize()
    say(f"  chosen blocks per CU {bpc}, open lanes {lanes}, slabs {slabs}")
    assert bpc in (4, 8, 16) and lanes in (0, 8, 16, 32, 48) and slabs in (0, 1)
    k = n * W
    for U, D in ((U1, D1), (U2, D2)):
        assert torch.equal(U[:k], U0[:k]) and torch.equal(D[:k], D0[:k])
    assert torch.equal(rec2["exit"][:, :k], rec0["exit"][:, :k])
    assert torch.equal(c2[1:], c0[1:]) and torch.equal(c1[1:], c0[1:])


@pytest.mark.parametrize("dim", [2, 3])
def test_tuned_pointwise_walks_are_bit_identical(dim):
    _bvc, pl = lib()
    say(f"tune pointwise walks dim={dim}")
    if dim == 2:
        scene = small_star()
        g, f = c2_like_fields()
        fd = pl.DeviceField(f)
    else:
        scene = wl.displaced_icosphere(3, 31)
        g = wl.solid_harmonics_3d(np.random.default_rng(1).normal(0, 1, 16), 3)
        fd = None
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    osc_pts = wl.uniform_box(3000, np.array(scene.bbox[0]) * 0.5, np.array(scene.bbox[1]) * 0.5, 5)
    x = torch.from_numpy(np.ascontiguousarray(osc_pts.T)).to("cuda", torch.float32)
    n, W = x.shape[1], 16
    params = pl.walk_params(3e-3, W, 79, gd, fd, "f32")
    u0, g0, c0 = pl.pointwise(sc, params, x, with_grad=True)
    Uw = torch.empty(n * W, dtype=torch.float32, device="cuda")
    Gw = torch.empty(dim, n * W, dtype=torch.float32, device="cuda")
    work = torch.empty(_bvc.bvc_pointwise_workspace_bytes(dim, n, W, _bvc.F32, True), dtype=torch.uint8, device="cuda")
    u1, g1 = torch.empty_like(u0), torch.empty_like(g0)
    c1 = torch.zeros(4, dtype=torch.int64, device="cuda")
    bpc, lanes, slabs = _bvc.bvc_tune_pointwise(sc.h, params, n, x, Uw, Gw, work, u1, g1, c1, reps=1)
    u2, g2, c2 = pl.pointwise(sc, params, x, with_grad=True)
    torch.cuda.synchronize()
    say(f"  chosen blocks per CU {bpc}, open lanes {lanes}, slabs {slabs}")
    assert bpc in (4, 8, 16) and lanes in (0, 8, 16, 32, 48) and slabs in ((0,) if dim == 2 else (0, 1))
    for u, gr in ((u1, g1), (u2, g2)):
        assert torch.equal(u, u0) and torch.equal(gr, g0)
    assert torch.equal(c2[1:], c0[1:]) and torch.equal(c1[1:], c0[1:])
