"""Edge cases of the HIP path through the C-ABI (marked gpu): empty inputs,
ragged sizes, the step cap, coincident points, a near field that covers the
whole scene, and the smallest scenes (a triangle, a tetrahedron).  Each result
is compared with the oracle or with what the method fixes for that case."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import abs_terms, lib, oracle_cache, per_walk_match, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _views(_bvc, T, code, cy, cn, a, b, sy=None, sw=None):
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", T)
    cache = dict(n=cy.shape[0], dtype=code, x=dev(cy), nrm=dev(cn), a=dev(a), b=dev(b))
    src = None if sy is None else dict(n=sy.shape[0], dtype=code, y=dev(sy), s=dev(sw))
    return cache, src, dev


@pytest.mark.parametrize("dim", [2, 3])
def test_gather_empty_inputs(orc, dim):
    _bvc, pl = lib()
    say(f"gather empty inputs dim={dim}")
    rng = np.random.default_rng(3)
    T, code = torch.float64, _bvc.F64
    sy = rng.uniform(-0.5, 0.5, (37, dim))
    sw = rng.normal(0, 1, 37)
    empty = np.zeros((0, dim))
    cache, src, dev = _views(_bvc, T, code, empty, empty, np.zeros(0), np.zeros(0), sy, sw)
    # no evaluation points: nothing is written
    u = torch.full((4,), 7.0, dtype=T, device="cuda")
    _bvc.bvc_gather_u(dim, cache, src, 0, dev(np.zeros((1, dim))), u)
    torch.cuda.synchronize()
    assert torch.all(u == 7.0)
    # no cache points: the source term alone (Eq. 4)
    x = rng.uniform(-0.9, 0.9, (29, dim))
    g = torch.empty(dim, 29, dtype=T, device="cuda")
    u = torch.empty(29, dtype=T, device="cuda")
    _bvc.bvc_gather_grad(dim, cache, src, 29, dev(x), u, g)
    torch.cuda.synchronize()
    uo, go = orc.gather(dim, x, empty, empty, np.zeros(0), np.zeros(0), sy, sw)
    assert np.allclose(u.cpu().numpy(), uo, rtol=1e-12, atol=1e-14)
    assert np.allclose(to_np_aos(g), go, rtol=1e-12, atol=1e-12)
    # neither cache nor sources: zero, and accumulate leaves the values
    u0 = torch.zeros(29, dtype=T, device="cuda")
    _bvc.bvc_gather_u(dim, cache, None, 29, dev(x), u0)
    u1 = torch.full((29,), 2.5, dtype=T, device="cuda")
    _bvc.bvc_gather_u(dim, cache, None, 29, dev(x), u1, accumulate=1)
    torch.cuda.synchronize()
    assert torch.all(u0 == 0) and torch.all(u1 == 2.5)


def test_walks_empty_inputs():
    _bvc, pl = lib()
    say("walks with no start points")
    sc = pl.Scene(wl.circle_polygon(64))
    g = pl.DeviceField(wl.harmonic_2d(3, 1.0, 1.0))
    params = pl.walk_params(1e-3, 16, 5, g, None, "f32")
    cache = pl.sample_cache(sc, 0, 5e-3, 1, 3, 0)
    assert cache.n == 0
    U, D, rec, counters = pl.cache_walks(sc, cache, params, "f32")
    uhat, dudn, a, b = pl.reduce_walks(cache, 16, U, D, "f32")
    u, gr, cnt = pl.pointwise(sc, params, torch.zeros(2, 0, device="cuda"), with_grad=True)
    torch.cuda.synchronize()
    assert counters.cpu().numpy().tolist() == [0, 0, 0, 0]
    assert cnt.cpu().numpy()[1:].tolist() == [0, 0, 0]


def test_step_cap_of_one(orc):
    """max_steps = 1: a walk ends at its first query, inside the shell or
    capped there, and reads g at that query's closest point (Section 3.1 with
    the cap of the readings).  FP64, walk by walk against the oracle."""
    _bvc, pl = lib()
    say("step cap of one")
    scene, g = wl.circle_polygon(128), wl.harmonic_2d(3, 1.0, 1.0)
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    cache = pl.sample_cache(sc, 300, 5e-3, 1, 8, 0)
    W = 8
    params = pl.walk_params(1e-3, W, 31, gd, None, "f64", max_steps=1)
    U, D, rec, counters = pl.cache_walks(sc, cache, params, "f64", records=True)
    torch.cuda.synchronize()
    cn = oracle_cache(orc.Scene(scene).sample_cache(300, 5e-3, 1, 8, 0), cache)
    ref = orc.cache_walks(orc.Scene(scene), g, None, orc.walk_params(1e-3, W, 31, max_steps=1), cn)
    n = cache.n * W
    assert np.all(rec["steps"].cpu().numpy()[:n] == 1)
    assert per_walk_match(U.cpu().numpy()[:n], ref["U"]).mean() >= 0.999
    assert per_walk_match(D.cpu().numpy()[:n], ref["D"]).mean() >= 0.999
    c = counters.cpu().numpy()
    # every walk whose first query lies outside the shell is capped
    assert c[1] == n and 0 < c[2] <= n


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_gather_coincident_point_is_finite(dtype):
    """An evaluation point on a cache point: the pair's 1/r^2 terms are
    singular; the kernel keeps r^2 + tiny and the result stays finite."""
    _bvc, pl = lib()
    say(f"gather coincident point {dtype}")
    rng = np.random.default_rng(5)
    T, code = (torch.float32, _bvc.F32) if dtype == "f32" else (torch.float64, _bvc.F64)
    th = rng.uniform(0, 2 * np.pi, 300)
    cy = np.stack([np.cos(th), np.sin(th)], 1)
    cache, _, dev = _views(_bvc, T, code, cy, cy.copy(), rng.normal(0, 1, 300) / 300, rng.normal(0, 1, 300) / 300)
    x = np.concatenate([cy[:3], rng.uniform(-0.5, 0.5, (5, 2))])
    u = torch.empty(8, dtype=T, device="cuda")
    g = torch.empty(2, 8, dtype=T, device="cuda")
    _bvc.bvc_gather_grad(2, cache, None, 8, dev(x), u, g)
    torch.cuda.synchronize()
    assert torch.isfinite(u).all() and torch.isfinite(g).all()


@pytest.mark.parametrize("dim", [2, 3])
def test_near_field_covering_the_scene_is_the_fp64_sum(orc, dim):
    """With tau larger than the scene every boundary pair takes the FP64 near
    path: the FP32 gather then returns the FP64 sum (Eqs. 3 and 5), rounded
    once to FP32."""
    _bvc, pl = lib()
    say(f"near field covering the scene dim={dim}")
    rng = np.random.default_rng(7 + dim)
    N, K = 700, 333
    d = rng.normal(0, 1, (N, dim))
    cy = d / np.linalg.norm(d, axis=1, keepdims=True)
    cy32 = cy.astype(np.float32).astype(np.float64)
    a = (rng.normal(0, 1, N) / N).astype(np.float32).astype(np.float64)
    b = (rng.normal(0, 1, N) / N).astype(np.float32).astype(np.float64)
    x = rng.uniform(-0.6, 0.6, (K, dim))
    cache, _, dev = _views(_bvc, torch.float32, _bvc.F32, cy32, cy32, a, b)
    D = torch.float64
    d64 = lambda v: torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", D)
    near = dict(tau=10.0, x=d64(x), cx=d64(cy32), cn=d64(cy32), a=d64(a), b=d64(b))
    u = torch.empty(K, dtype=torch.float32, device="cuda")
    g = torch.empty(dim, K, dtype=torch.float32, device="cuda")
    _bvc.bvc_gather_grad(dim, cache, None, K, dev(x), u, g, near=near)
    torch.cuda.synchronize()
    uo, go, cond = orc.gather(dim, x, cy32, cy32, a, b, with_grad=True, with_cond=True)
    uu = 2.0**-24
    assert np.all(np.abs(u.double().cpu().numpy() - uo) <= uu * np.abs(uo) + 1e-12 * cond)
    gd = to_np_aos(g)
    assert np.all(np.abs(gd - go) <= uu * np.abs(go) + 1e-11 * (np.abs(go).max() + cond.max()))


@pytest.mark.parametrize("dim", [2, 3])
def test_near_field_lead(orc, dim):
    """Evaluation points that can meet a cache point closer than tau ordered
    first, their count passed as near_lead: the blocks past them skip the
    near test.  The leading points (near path in both launches) agree bit for
    bit with a launch that tests every point, the trailing ones (no pair
    closer than tau) to FP32 rounding of the sum of |terms|; a lead outside
    [0, n_eval] is refused."""
    _bvc, pl = lib()
    say(f"near field lead dim={dim}")
    rng = np.random.default_rng(31 + dim)
    N, n_near, n_far = 700, 1301, 3790
    d = rng.normal(0, 1, (N, dim))
    cy = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    a = (rng.normal(0, 1, N) / N).astype(np.float32).astype(np.float64)
    b = (rng.normal(0, 1, N) / N).astype(np.float32).astype(np.float64)
    tau = 0.05
    # leading points 0.02 inside a cache point, trailing ones at radius <= 0.8
    xn = cy[np.arange(n_near) % N] * 0.98
    xf = rng.normal(0, 1, (n_far, dim))
    xf *= rng.uniform(0, 0.8, (n_far, 1)) / np.linalg.norm(xf, axis=1, keepdims=True)
    x = np.concatenate([xn, xf])
    K = x.shape[0]
    cache, _, dev = _views(_bvc, torch.float32, _bvc.F32, cy, cy, a, b)
    d64 = lambda v: torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", torch.float64)
    near = dict(tau=tau, x=d64(x), cx=d64(cy), cn=d64(cy), a=d64(a), b=d64(b))
    out = []
    for lead in (0, n_near):
        u = torch.empty(K, dtype=torch.float32, device="cuda")
        g = torch.empty(dim, K, dtype=torch.float32, device="cuda")
        _bvc.bvc_gather_grad(dim, cache, None, K, dev(x), u, g, near=dict(near, lead=lead))
        torch.cuda.synchronize()
        out.append((u.double().cpu().numpy(), to_np_aos(g)))
    (u0, g0), (u1, g1) = out
    assert np.array_equal(u1[:n_near], u0[:n_near]) and np.array_equal(g1[:n_near], g0[:n_near])
    # (one source of weight 0 far away: abs_terms wants a source)
    su, sun, sg, sgn, _ = abs_terms(dim, xf, cy, cy, a, b, np.full((1, dim), 10.0), np.zeros(1), tau)
    assert np.all(sun == 0) and np.all(sgn == 0)
    uu = 2.0**-24
    assert np.all(np.abs(u1[n_near:] - u0[n_near:]) <= 64 * uu * su)
    assert np.all(np.abs(g1[n_near:] - g0[n_near:]) <= 64 * uu * sg[:, None])
    u = torch.empty(K, dtype=torch.float32, device="cuda")
    for lead in (-1, K + 1):
        with pytest.raises(_bvc.BVCError):
            _bvc.bvc_gather_u(dim, cache, None, K, dev(x), u, near=dict(near, lead=lead))


@pytest.mark.parametrize("n_cand", [1, 7, 4097])
def test_sampler_ragged_counts(orc, n_cand):
    _bvc, pl = lib()
    say(f"sampler ragged n={n_cand}")
    scene = wl.circle_polygon(64)
    sc = pl.Scene(scene)
    d = 2
    f64 = torch.float64
    x = torch.empty(d, n_cand, dtype=f64, device="cuda")
    nrm, xbar = torch.empty_like(x), torch.empty_like(x)
    w = torch.empty(n_cand, dtype=f64, device="cuda")
    R0 = torch.empty_like(w)
    acc = torch.empty(n_cand, dtype=torch.int32, device="cuda")
    _bvc.bvc_sample_cache(sc.h, n_cand, 5e-3, 1, 19, 0, x, nrm, w, xbar, R0, acc)
    torch.cuda.synchronize()
    ref = orc.Scene(scene).sample_cache(n_cand, 5e-3, 1, 19)
    assert np.array_equal(acc.cpu().numpy().astype(bool), ref["accept"])
    m = ref["accept"]
    assert np.allclose(to_np_aos(x)[m], ref["x"][m], rtol=0, atol=1e-13)


@pytest.mark.parametrize("which", ["triangle", "tetrahedron"])
def test_smallest_scenes(orc, which):
    """A single-leaf-sized scene (3 segments, 4 triangles): BVH root with
    primitive leaves, walks and their means against the oracle, walk by walk."""
    _bvc, pl = lib()
    say(f"smallest scene {which}")
    if which == "triangle":
        verts = np.array([[0.0, 0.0], [1.0, 0.0], [0.2, 0.9]])
        prims = np.array([[0, 1], [1, 2], [2, 0]], dtype=np.int32)
        g = wl.harmonic_2d(3, 1.0, 1.0)
    else:
        verts = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
        prims = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)
        g = wl.solid_harmonics_3d(np.random.default_rng(2).normal(0, 1, 81), 8)
    scene = wl.Scene(verts.shape[1], verts, prims, which)
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    l = 0.02
    cache = pl.sample_cache(sc, 400, l, 1, 4, 0)
    assert cache.n > 0
    W = 16
    params = pl.walk_params(2e-3, W, 13, gd, None, "f64")
    U, D, rec, counters = pl.cache_walks(sc, cache, params, "f64")
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    ref = orc.cache_walks(osc, g, None, orc.walk_params(2e-3, W, 13), oracle_cache(osc.sample_cache(400, l, 1, 4, 0), cache))
    n = cache.n * W
    assert per_walk_match(U.cpu().numpy()[:n], ref["U"]).mean() >= 0.999
    assert per_walk_match(D.cpu().numpy()[:n], ref["D"]).mean() >= 0.999
