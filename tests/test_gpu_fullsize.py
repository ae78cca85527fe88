"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (marked gpu).  The whole step runs at its real shape; the oracle then
recomputes sampled outputs one by one from its own inputs (its own
classification, cache and sources, each first checked equal to the
device's; the gather kernel is launched at full size on the oracle's cache
with seeded cache values):

- C2 (4096-segment star, 16,384 cache points x 256 walks, 1024^2 grid) in
  FP64: per-walk parity of every walk of 24 cache points spread over the
  cache; u and grad u at 64 interior points of a full-size gather against
  the oracle's gather over the whole cache and source set; the 256 walks of 32 band points replayed
  walk by walk (same ids, same Philox streams).
- C2 in FP32, as timed (FP64 near field for pairs closer than l): per-point
  walk means of 16 cache points against the oracle's FP64 walks on the same
  streams (3 sigma), u and grad u at 64 interior points of a full-size FP32
  gather with the near field on the oracle's cache and sources within the
  FP32 bound of the far pairs, band means against the oracle's walks.
- C3 (displaced icosphere, 65,536 x 512 walks, 1.1 M points) in FP32, as
  timed: per-point walk means of 16 cache points and 16 band points against
  the oracle's FP64 walks on the same streams (z-test), and u at 64 interior
  points of a full-size FP32 gather against the oracle's within the FP32
  error bound.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import abs_terms, lib, oracle_cache, per_walk_match, to_np_aos, z_ok

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _spread(n, k):
    return np.unique(np.linspace(0, n - 1, min(k, n)).astype(np.int64))


def _band_walks(orc, osc, prob, params, pts, band_index, W, with_grad):
    """Mean of the W pointwise walks of each band point, walk ids k*W + j as
    the library numbers the band points (k = index in the band set)."""
    d, xb, _ = osc.closest(pts)
    u = np.zeros(len(pts))
    g = np.zeros((len(pts), prob.scene.dim))
    se = np.zeros(len(pts))
    for i, k in enumerate(band_index):
        us, gs = [], []
        for j in range(W):
            w = orc.walk(osc, prob.g, prob.f, params, 1, pts[i], None, d[i], xb[i], int(k) * W + j)
            us.append(w["U"])
            gs.append(w["grad"])
        us = np.array(us)
        u[i] = us.mean()
        se[i] = us.std() / np.sqrt(W)
        g[i] = np.mean(gs, axis=0)
    return u, g, se


def _dev(v, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", dtype)


def _oracle_split(osc, prob, prep):
    """The oracle's interior and band index sets; the device's must equal them."""
    cls = osc.classify(prob.eval_x, prob.offset)
    idx_i, idx_b = np.flatnonzero(cls == 1), np.flatnonzero(cls == 2)
    assert np.array_equal(prep.idx_int[: prep.n_int].cpu().numpy(), idx_i)
    assert np.array_equal(prep.idx_band[: prep.n_band].cpu().numpy(), idx_b)
    return idx_i, idx_b


def _cache_values(cn, seed):
    """Seeded cache values a, b for a gather launched on the oracle's cache."""
    rng = np.random.default_rng(seed)
    n = cn["x"].shape[0]
    return rng.normal(0, 1, n) * cn["w"], rng.normal(0, 1, n) * cn["w"]


def test_c2_full_size_fp64(orc):
    _bvc, pl = lib()
    prob = wl.problem_c2()
    say("c2 full size fp64: prepare")
    prep = pl.Prepared(prob, dtype="f64")
    W = prob.n_walks
    sol = pl.solve(prep, batch=0, with_grad=True)
    torch.cuda.synchronize()
    cache = sol.cache
    n = cache.n
    say(f"c2 full size fp64: cache {n} interior {prep.n_int} band {prep.n_band}")
    assert 14000 <= n <= 19000 and prep.n_int > 400000 and prep.n_band > 50000
    c = sol.counters.cpu().numpy()
    assert c[3] == n * W and c[2] == 0
    osc = orc.Scene(prob.scene)
    P = orc.walk_params(prob.eps, W, prob.seed_walks)
    idx_i, idx_b = _oracle_split(osc, prob, prep)
    cn = oracle_cache(osc.sample_cache(prep.n_cand, prob.offset, prob.sides, prob.seed_cache, 0), cache)
    # walks of 24 cache points, walk by walk
    pick = _spread(n, 24)
    ids = (pick[:, None] * W + np.arange(W)[None, :]).ravel()
    ref = orc.cache_walks_subset(osc, prob.g, prob.f, P, cn, ids)
    Ug = sol.extra["U"].cpu().numpy()[ids]
    Dg = sol.extra["D"].cpu().numpy()[ids]
    okU, okD = per_walk_match(Ug, ref["U"]), per_walk_match(Dg, ref["D"])
    say(f"  walks {ids.size}: U-match {okU.mean():.5f} D-match {okD.mean():.5f}")
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999
    # the oracle's sources; the device's must be the same
    m = int(round(prob.n_sources ** 0.5))
    lo, hi = prob.scene.bbox
    sy, sw = osc.sample_sources(prob.f, m, lo, hi, prob.offset, prob.seed_sources, 0)
    sv = sol.extra["sview"]
    assert sv["n"] == sw.size
    assert np.allclose(to_np_aos(sv["y"], sv["n"]), sy, rtol=0, atol=1e-13)
    assert np.allclose(sv["s"].cpu().numpy()[: sv["n"]], sw, rtol=1e-12, atol=0)
    # a full-size gather (every interior point, the whole cache and source
    # set, as the step launches it) on the oracle's cache with seeded values;
    # 64 of its outputs against the oracle's gather
    a, b = _cache_values(cn, 5)
    cview = dict(n=n, dtype=_bvc.F64, x=_dev(cn["x"]), nrm=_dev(cn["n"]), a=_dev(a), b=_dev(b))
    sview = dict(n=sw.size, dtype=_bvc.F64, y=_dev(sy), s=_dev(sw))
    u_full = torch.empty(prep.n_int, dtype=torch.float64, device="cuda")
    g_full = torch.empty(2, prep.n_int, dtype=torch.float64, device="cuda")
    _bvc.bvc_gather_grad(2, cview, sview, prep.n_int, _dev(prob.eval_x[idx_i]), u_full, g_full)
    torch.cuda.synchronize()
    ki = _spread(prep.n_int, 64)
    x = prob.eval_x[idx_i[ki]]
    uo, go, cond = orc.gather(2, x, cn["x"], cn["n"], a, b, sy, sw, with_grad=True, with_cond=True)
    ug = u_full.cpu().numpy()[ki]
    gg = to_np_aos(g_full)[ki]
    assert np.all(np.abs(ug - uo) <= 1e-11 * cond)
    gsc = np.abs(go).max(1) + cond
    assert np.all(np.abs(gg - go).max(1) <= 1e-9 * gsc)
    # the step's own estimate is close to the solution
    tru = wl.field_value(prob.truth, prob.eval_x[idx_i])
    err = np.median(np.abs(sol.u_int.cpu().numpy()[: prep.n_int] - tru))
    say(f"  interior median error {err:.4g}")
    assert err < 0.02 * np.sqrt(np.mean(tru**2))
    # band points: the library's 256 walks per point, replayed walk by walk
    kb = _spread(prep.n_band, 32)
    pts = prob.eval_x[idx_b[kb]]
    ub, gb, se = _band_walks(orc, osc, prob, P, pts, kb, W, True)
    u_gpu = sol.u_band.cpu().numpy()[kb]
    g_gpu = to_np_aos(sol.g_band)[kb]
    close = per_walk_match(u_gpu, ub, 1e-9)
    say(f"  band points {kb.size}: mean-match {close.mean():.3f}")
    assert close.mean() >= 0.9
    assert np.all(np.abs(u_gpu - ub) <= 6 * se + 1e-12)
    assert np.mean(np.all(np.abs(g_gpu - gb) <= 1e-8 * (np.abs(gb) + 1), axis=1)) >= 0.9


def test_c2_full_size_fp32(orc):
    _bvc, pl = lib()
    prob = wl.problem_c2()
    say("c2 full size fp32: prepare")
    prep = pl.Prepared(prob, dtype="f32")
    assert prep.near_tau == prob.offset
    W = prob.n_walks
    sol = pl.solve(prep, batch=0, with_grad=True)
    torch.cuda.synchronize()
    cache = sol.cache
    n = cache.n
    say(f"c2 full size fp32: cache {n} interior {prep.n_int} band {prep.n_band}")
    assert 14000 <= n <= 19000 and prep.n_int > 400000 and prep.n_band > 50000
    c = sol.counters.cpu().numpy()
    assert c[3] == n * W and c[2] == 0
    osc = orc.Scene(prob.scene)
    P = orc.walk_params(prob.eps, W, prob.seed_walks)
    idx_i, idx_b = _oracle_split(osc, prob, prep)
    cn = oracle_cache(osc.sample_cache(prep.n_cand, prob.offset, prob.sides, prob.seed_cache, 0), cache)
    # walk means of 16 cache points against the FP64 walks on the same streams
    pick = _spread(n, 16)
    ids = (pick[:, None] * W + np.arange(W)[None, :]).ravel()
    ref = orc.cache_walks_subset(osc, prob.g, prob.f, P, cn, ids)
    for name in ("U", "D"):
        A = sol.extra[name].double().cpu().numpy()[ids].reshape(-1, W)
        Bo = ref[name].reshape(-1, W)
        se = np.sqrt(A.var(1, ddof=1) / W + Bo.var(1, ddof=1) / W) + 1e-12
        z = np.abs(A.mean(1) - Bo.mean(1)) / se
        ok, msg = z_ok(z)
        say(f"  {name}: {msg}")
        assert ok, msg
    # the oracle's sources; the device's must be the same
    m = int(round(prob.n_sources ** 0.5))
    lo, hi = prob.scene.bbox
    sy, sw = osc.sample_sources(prob.f, m, lo, hi, prob.offset, prob.seed_sources, 0)
    sv = sol.extra["sview"]
    assert sv["n"] == sw.size
    assert np.allclose(to_np_aos(sv["y"], sv["n"]), sy, rtol=0, atol=1e-6)
    # (FP32 weights: Gaussian tails below the FP32 range round to 0)
    assert np.allclose(sv["s"].double().cpu().numpy()[: sv["n"]], sw, rtol=1e-6, atol=1e-7 * np.abs(sw).max())
    # a full-size FP32 gather of u and grad u with the near field, as the
    # step launches it, on the oracle's cache and sources with seeded values
    # rounded to FP32 (the near field's FP64 copies hold the same numbers);
    # 64 outputs against the oracle
    r32 = lambda v: v.astype(np.float32).astype(np.float64)
    a, b = _cache_values(cn, 7)
    cy, cnn, a, b, sy, sw = (r32(v) for v in (cn["x"], cn["n"], a, b, sy, sw))
    xall = prob.eval_x[idx_i]
    f32, f64 = torch.float32, torch.float64
    tau = prep.near_tau
    cview = dict(n=n, dtype=_bvc.F32, x=_dev(cy, f32), nrm=_dev(cnn, f32), a=_dev(a, f32), b=_dev(b, f32))
    sview = dict(n=sw.size, dtype=_bvc.F32, y=_dev(sy, f32), s=_dev(sw, f32))
    near = dict(tau=tau, x=_dev(xall, f64), cx=_dev(cy, f64), cn=_dev(cnn, f64), a=_dev(a, f64), b=_dev(b, f64))
    u_full = torch.empty(prep.n_int, dtype=f32, device="cuda")
    g_full = torch.empty(2, prep.n_int, dtype=f32, device="cuda")
    _bvc.bvc_gather_grad(2, cview, sview, prep.n_int, _dev(xall, f32), u_full, g_full, near=near)
    torch.cuda.synchronize()
    ki = _spread(prep.n_int, 64)
    x = xall[ki]
    uo, go = orc.gather(2, x, cy, cnn, a, b, sy, sw, with_grad=True)
    su_far, su_near, sg_far, sg_near, rmin = abs_terms(2, x, cy, cnn, a, b, sy, sw, tau)
    uu = 2.0**-24
    zmax = np.linalg.norm(np.concatenate([cy, sy]), axis=1).max()
    x32 = r32(x)
    shift = np.linalg.norm(x - x32, axis=1) / rmin
    rel = uu * (300 + 4 * (np.linalg.norm(x, axis=1) + zmax) / rmin) + 4 * shift
    tol = su_far * rel + 1e-10 * su_near + uu * np.abs(uo)
    err = np.abs(u_full.double().cpu().numpy()[ki] - uo)
    assert np.all(err <= tol), np.max(err / tol)
    gtol = sg_far * (rel + 2 * shift) + 1e-10 * sg_near + uu * np.abs(go).max(1)
    gerr = np.abs(to_np_aos(g_full)[ki] - go).max(1)
    assert np.all(gerr <= gtol + 1e-30), np.max(gerr / gtol)
    # the step's own estimate is close to the solution
    tru = wl.field_value(prob.truth, xall)
    err = np.median(np.abs(sol.u_int.double().cpu().numpy()[: prep.n_int] - tru))
    say(f"  interior median error {err:.4g}")
    assert err < 0.02 * np.sqrt(np.mean(tru**2))
    # band points: walk means against the FP64 walks on the same streams
    kb = _spread(prep.n_band, 16)
    pts = prob.eval_x[idx_b[kb]]
    ub, _, se_o = _band_walks(orc, osc, prob, P, pts, kb, W, True)
    u_gpu = sol.u_band.double().cpu().numpy()[kb]
    z = np.abs(u_gpu - ub) / (np.sqrt(2) * se_o + 1e-6 * (1 + np.abs(ub)))
    ok, msg = z_ok(z)
    say(f"  band: {msg}")
    assert ok, msg


def test_c3_full_size_fp32(orc):
    _bvc, pl = lib()
    prob = wl.problem_c3()
    say("c3 full size fp32: prepare")
    prep = pl.Prepared(prob, dtype="f32")
    W = prob.n_walks
    sol = pl.solve(prep, batch=0, with_grad=False)
    torch.cuda.synchronize()
    cache = sol.cache
    n = cache.n
    say(f"c3 full size fp32: cache {n} interior {prep.n_int} band {prep.n_band}")
    assert 60000 <= n <= 72000 and prep.n_int > 1_000_000
    c = sol.counters.cpu().numpy()
    assert c[3] == n * W and c[2] == 0
    osc = orc.Scene(prob.scene)
    P = orc.walk_params(prob.eps, W, prob.seed_walks)
    idx_i, idx_b = _oracle_split(osc, prob, prep)
    cn = oracle_cache(osc.sample_cache(prep.n_cand, prob.offset, prob.sides, prob.seed_cache, 0), cache)
    # walk means of 16 cache points against the FP64 walks on the same streams
    pick = _spread(n, 16)
    ids = (pick[:, None] * W + np.arange(W)[None, :]).ravel()
    ref = orc.cache_walks_subset(osc, prob.g, None, P, cn, ids)
    for name in ("U", "D"):
        A = sol.extra[name].double().cpu().numpy()[ids].reshape(-1, W)
        Bo = ref[name].reshape(-1, W)
        se = np.sqrt(A.var(1) / W + Bo.var(1) / W) + 1e-12
        z = np.abs(A.mean(1) - Bo.mean(1)) / se
        say(f"  {name}: max z {z.max():.2f}")
        assert np.all(z < 5)
    # a full-size FP32 gather (every interior point, the whole cache) on the
    # oracle's cache with seeded values, all rounded to FP32 on the host; 64
    # of its outputs against the oracle's gather of the rounded inputs
    r32 = lambda v: v.astype(np.float32).astype(np.float64)
    a, b = _cache_values(cn, 6)
    cy, cnn, a, b = r32(cn["x"]), r32(cn["n"]), r32(a), r32(b)
    xall = r32(prob.eval_x[idx_i])
    f32 = torch.float32
    cview = dict(n=n, dtype=_bvc.F32, x=_dev(cy, f32), nrm=_dev(cnn, f32), a=_dev(a, f32), b=_dev(b, f32))
    u_full = torch.empty(prep.n_int, dtype=f32, device="cuda")
    _bvc.bvc_gather_u(3, cview, None, prep.n_int, _dev(xall, f32), u_full)
    torch.cuda.synchronize()
    ki = _spread(prep.n_int, 64)
    x = xall[ki]
    uo, cond = orc.gather(3, x, cy, cnn, a, b, with_grad=False, with_cond=True)
    ug = u_full.double().cpu().numpy()[ki]
    rmin = np.min(np.linalg.norm(x[:, None, :] - cy[None], axis=2), axis=1)
    zmax = np.linalg.norm(cy, axis=1).max()
    uu = 2.0**-24
    tol = uu * cond * (300 + 4 * (np.linalg.norm(x, axis=1) + zmax) / rmin) + uu * np.abs(uo)
    assert np.all(np.abs(ug - uo) <= tol), np.max(np.abs(ug - uo) / tol)
    # the step's own estimate is close to the solution
    tru = wl.field_value(prob.truth, prob.eval_x[idx_i])
    err = np.median(np.abs(sol.u_int.double().cpu().numpy()[: prep.n_int] - tru))
    say(f"  interior median error {err:.4g}")
    # (degree-8 solid harmonics on the displaced sphere: a median error of about
    # 4% of the RMS of u with 512 walks per cache point)
    assert err < 0.1 * np.sqrt(np.mean(tru**2))
    # band points: walk means against the FP64 walks on the same streams
    kb = _spread(prep.n_band, 16)
    pts = prob.eval_x[idx_b[kb]]
    ub, _, se_o = _band_walks(orc, osc, prob, P, pts, kb, W, False)
    u_gpu = sol.u_band.double().cpu().numpy()[kb]
    # points inside the epsilon shell return g at their closest point on every
    # walk (zero spread): there the FP32 rounding of the result is the bound
    z = np.abs(u_gpu - ub) / (np.sqrt(2) * se_o + 1e-6 * (1 + np.abs(ub)))
    say(f"  band: max z {z.max():.2f}, shell points {int(np.sum(se_o == 0))}")
    assert np.all(z < 5)
