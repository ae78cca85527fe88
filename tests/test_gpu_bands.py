"""Bands of pointwise walks next to the boundary (marked gpu), FP64 against
the oracle on the same Philox streams.

- Gradient band: gathered points within w of the boundary take grad u from
  pointwise walks (the gradient estimate of Eq. 7 at the point) and keep the
  gathered u.  The points chosen are the oracle's (interior at l, inside w),
  u and grad u elsewhere are bit for bit those of the solve without the band,
  and the replaced gradients are the oracle's pointwise means on the walk ids
  k W + j of the band's k-th point with the gradient band's batch word.
- Wide band: points within w > l take pointwise u and grad u; the band is the
  oracle's classification at w and its values are the oracle's pointwise
  means.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import c2_like_fields, lib, per_walk_match, small_star, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _problem():
    sc = small_star()
    g, f = c2_like_fields()
    lo, hi = sc.bbox
    eps = 3e-3
    return wl.Problem("star512_bands", sc, g, f, 2048, 16, eps, 5 * eps, 1024, wl.grid2d(96, lo, hi), g, sides=2,
                      precision="f64", seed_walks=77, seed_cache=78, seed_sources=79)


def test_grad_band_fp64(orc):
    _bvc, pl = lib()
    prob = _problem()
    l, W = prob.offset, prob.n_walks
    width = 4 * l
    say(f"grad band fp64: width {width}")
    p0 = pl.Prepared(prob, dtype="f64")
    p1 = pl.Prepared(prob, dtype="f64", n_cand=p0.n_cand, grad_band=width)
    s0 = pl.solve(p0, batch=3, with_grad=True)
    s1 = pl.solve(p1, batch=3, with_grad=True)
    torch.cuda.synchronize()
    osc = orc.Scene(prob.scene)
    idx_i = p0.idx_int[: p0.n_int].cpu().numpy()
    xi = prob.eval_x[idx_i]
    want = np.flatnonzero(osc.classify(xi, width) == 2)
    pos = p1.gb_pos[: p1.n_gb].cpu().numpy()
    assert p1.n_gb > 50 and np.array_equal(pos, want)
    u0, u1 = to_np_aos(s0.u_int, p0.n_int), to_np_aos(s1.u_int, p1.n_int)
    g0, g1 = to_np_aos(s0.g_int, p0.n_int), to_np_aos(s1.g_int, p1.n_int)
    assert np.array_equal(u0, u1)
    rest = np.ones(p0.n_int, bool)
    rest[pos] = False
    assert np.array_equal(g0[rest], g1[rest])
    P = orc.walk_params(prob.eps, W, prob.seed_walks, batch=3 | pl.GRAD_BAND_BATCH_BIT)
    _, go, _ = orc.pointwise(osc, prob.g, prob.f, P, xi[pos], with_grad=True)
    ok = per_walk_match(g1[pos], go, 1e-8).all(axis=1)
    say(f"  {pos.size} points, match {ok.mean():.4f}")
    assert ok.mean() >= 0.99
    # the gathered gradient next to the cache surface is what the band replaces
    assert not np.allclose(g0[pos], g1[pos])
    assert s1.extra["grad_band"]["n"] == pos.size


def test_wide_band_fp64(orc):
    _bvc, pl = lib()
    prob = _problem()
    l, W = prob.offset, prob.n_walks
    width = 2 * l
    say(f"wide band fp64: width {width}")
    p2 = pl.Prepared(prob, dtype="f64", band=width)
    s2 = pl.solve(p2, batch=5, with_grad=True)
    torch.cuda.synchronize()
    osc = orc.Scene(prob.scene)
    cls = osc.classify(prob.eval_x, width)
    assert np.array_equal(p2.idx_band[: p2.n_band].cpu().numpy(), np.flatnonzero(cls == 2))
    assert np.array_equal(p2.idx_int[: p2.n_int].cpu().numpy(), np.flatnonzero(cls == 1))
    pts = prob.eval_x[np.flatnonzero(cls == 2)]
    P = orc.walk_params(prob.eps, W, prob.seed_walks, batch=5)
    uo, go, _ = orc.pointwise(osc, prob.g, prob.f, P, pts, with_grad=True)
    oku = per_walk_match(to_np_aos(s2.u_band, p2.n_band), uo, 1e-9)
    okg = per_walk_match(to_np_aos(s2.g_band, p2.n_band), go, 1e-8).all(axis=1)
    say(f"  {pts.shape[0]} band points, match u {oku.mean():.4f} grad {okg.mean():.4f}")
    assert oku.mean() >= 0.99 and okg.mean() >= 0.99
