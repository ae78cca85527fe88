"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (marked gpu).  The whole step runs at its real shape; the oracle then
recomputes sampled outputs one by one on the same inputs:

- C2 (4096-segment star, 16,384 cache points x 256 walks, 1024^2 grid) in
  FP64: per-walk parity of every walk of 24 cache points spread over the
  cache; u and grad u at 64 interior points against the oracle's gather over
  the whole cache and source set; the 256 walks of 32 band points replayed
  walk by walk (same ids, same Philox streams).
- C3 (displaced icosphere, 65,536 x 512 walks, 1.1 M points) in FP32, as
  timed: per-point walk means of 16 cache points and 16 band points against
  the oracle's FP64 walks on the same streams (z-test), and u at 64 interior
  points against the oracle's gather within the FP32 error bound.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import cache_np, lib, per_walk_match, to_np_aos

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
    cn = cache_np(cache)
    # walks of 24 cache points, walk by walk
    pick = _spread(n, 24)
    ids = (pick[:, None] * W + np.arange(W)[None, :]).ravel()
    ref = orc.cache_walks_subset(osc, prob.g, prob.f, P, cn, ids)
    Ug = sol.extra["U"].cpu().numpy()[ids]
    Dg = sol.extra["D"].cpu().numpy()[ids]
    okU, okD = per_walk_match(Ug, ref["U"]), per_walk_match(Dg, ref["D"])
    say(f"  walks {ids.size}: U-match {okU.mean():.5f} D-match {okD.mean():.5f}")
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999
    # gather at 64 interior points over the whole cache and source set
    ki = _spread(prep.n_int, 64)
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    x = prob.eval_x[idx_i[ki]]
    a = sol.extra["a"].cpu().numpy()[:n]
    b = sol.extra["b"].cpu().numpy()[:n]
    sv = sol.extra["sview"]
    sy, sw = to_np_aos(sv["y"], sv["n"]), sv["s"].cpu().numpy()[: sv["n"]]
    uo, go, cond = orc.gather(2, x, cn["x"], cn["n"], a, b, sy, sw, with_grad=True, with_cond=True)
    ug = sol.u_int.cpu().numpy()[ki]
    gg = to_np_aos(sol.g_int)[ki]
    assert np.all(np.abs(ug - uo) <= 1e-11 * cond)
    gsc = np.abs(go).max(1) + cond
    assert np.all(np.abs(gg - go).max(1) <= 1e-9 * gsc)
    # band points: the library's 256 walks per point, replayed walk by walk
    kb = _spread(prep.n_band, 32)
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    pts = prob.eval_x[idx_b[kb]]
    ub, gb, se = _band_walks(orc, osc, prob, P, pts, kb, W, True)
    u_gpu = sol.u_band.cpu().numpy()[kb]
    g_gpu = to_np_aos(sol.g_band)[kb]
    close = per_walk_match(u_gpu, ub, 1e-9)
    say(f"  band points {kb.size}: mean-match {close.mean():.3f}")
    assert close.mean() >= 0.9
    assert np.all(np.abs(u_gpu - ub) <= 6 * se + 1e-12)
    assert np.mean(np.all(np.abs(g_gpu - gb) <= 1e-8 * (np.abs(gb) + 1), axis=1)) >= 0.9


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
    cn = cache_np(cache)
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
    # gather at 64 interior points (FP32 inputs as the device holds them)
    ki = _spread(prep.n_int, 64)
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    x = to_np_aos(prep.x_int)[ki]
    cv = sol.extra["cview"]
    cy, cnn = to_np_aos(cv["x"], n), to_np_aos(cv["nrm"], n)
    a = cv["a"].double().cpu().numpy()[:n]
    b = cv["b"].double().cpu().numpy()[:n]
    uo, cond = orc.gather(3, x, cy, cnn, a, b, with_grad=False, with_cond=True)
    ug = sol.u_int.double().cpu().numpy()[ki]
    rmin = np.min(np.linalg.norm(x[:, None, :] - cy[None], axis=2), axis=1)
    zmax = np.linalg.norm(cy, axis=1).max()
    uu = 2.0**-24
    tol = uu * cond * (300 + 4 * (np.linalg.norm(x, axis=1) + zmax) / rmin) + uu * np.abs(uo)
    assert np.all(np.abs(ug - uo) <= tol), np.max(np.abs(ug - uo) / tol)
    assert np.allclose(prob.eval_x[idx_i[ki]], x, atol=1e-6)
    # band points: walk means against the FP64 walks on the same streams
    kb = _spread(prep.n_band, 16)
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    pts = prob.eval_x[idx_b[kb]]
    ub, _, se_o = _band_walks(orc, osc, prob, P, pts, kb, W, False)
    u_gpu = sol.u_band.double().cpu().numpy()[kb]
    # points inside the epsilon shell return g at their closest point on every
    # walk (zero spread): there the FP32 rounding of the result is the bound
    z = np.abs(u_gpu - ub) / (np.sqrt(2) * se_o + 1e-6 * (1 + np.abs(ub)))
    say(f"  band: max z {z.max():.2f}, shell points {int(np.sum(se_o == 0))}")
    assert np.all(z < 5)
