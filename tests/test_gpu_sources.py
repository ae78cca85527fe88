"""Source terms the earlier paths left out (marked gpu): screened walks with a
source (Eq. 1 with sigma > 0 and f != 0) and the first ball's gradient source
term in 3D, against the FP64 oracle on the same Philox streams.

- FP64 cache walks walk by walk (U and D, >= 99.9% within 1e-9): screened
  with an exponential-plane source in 2D (circle) and 3D (displaced sphere),
  and the Laplace 3D walk with a source (its D now carries the gradient
  source term);
- FP64 pointwise walks with gradients (point means within 1e-9 / 1e-8);
- FP32 pointwise means against the oracle's on independent streams at 3
  standard errors, as often as a normal distribution allows;
- the whole screened step with a source (walks, sources in the screened
  gather, band walks) against the closed form u = e^(b.x).
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, oracle_cache, per_walk_match, to_np_aos, z_ok

pytestmark = pytest.mark.gpu

SIG = 9.0


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _case(dim, sigma):
    b = np.array([0.9, -0.6, 0.5])[:dim]
    scene = wl.circle_polygon(256) if dim == 2 else wl.displaced_icosphere(3, 31, amp=0.1)
    g = wl.exp_plane(1.0, b)
    f = wl.exp_plane(float(b @ b) - sigma, b)
    return scene, g, f, b


@pytest.mark.parametrize("dim,sigma", [(2, SIG), (3, SIG), (3, 0.0)])
def test_cache_walks_with_source_fp64(orc, dim, sigma):
    _bvc, pl = lib()
    scene, g, f, _ = _case(dim, sigma)
    say(f"cache walks fp64 with source dim={dim} sigma={sigma}")
    sc = pl.Scene(scene)
    gd, fd = pl.DeviceField(g), pl.DeviceField(f)
    n, W, l = 800, 16, 5e-3
    cache = pl.sample_cache(sc, n, l, 1, 77, 0)
    params = pl.walk_params(1e-3, W, 4243, gd, fd, "f64", sigma=sigma)
    U, D, rec, counters = pl.cache_walks(sc, cache, params, "f64", records=True)
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    cn = oracle_cache(osc.sample_cache(n, l, 1, 77, 0), cache)
    ref = orc.cache_walks(osc, g, f, orc.walk_params(1e-3, W, 4243, sigma=sigma), cn, records=True)
    k = cache.n * W
    okU = per_walk_match(U.cpu().numpy()[:k], ref["U"])
    okD = per_walk_match(D.cpu().numpy()[:k], ref["D"])
    say(f"  walks {k}: U {okU.mean():.5f} D {okD.mean():.5f}")
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999
    assert np.mean(rec["steps"].cpu().numpy()[:k] == ref["steps"]) >= 0.999


def _interior(orc, scene, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = scene.bbox
    osc = orc.Scene(scene)
    out = []
    while len(out) < n:
        x = rng.uniform(lo, hi, (4 * n, scene.dim))
        d, _, _ = osc.closest(x)
        out.extend(x[(osc.inside(x) != 0) & (d > 2e-3)])
    return np.array(out[:n])


@pytest.mark.parametrize("dim,sigma", [(2, SIG), (3, SIG), (3, 0.0)])
def test_pointwise_with_source_fp64(orc, dim, sigma):
    _bvc, pl = lib()
    scene, g, f, _ = _case(dim, sigma)
    say(f"pointwise fp64 with source dim={dim} sigma={sigma}")
    sc = pl.Scene(scene)
    gd, fd = pl.DeviceField(g), pl.DeviceField(f)
    pts = _interior(orc, scene, 150, 5)
    W = 16
    params = pl.walk_params(1e-3, W, 99, gd, fd, "f64", sigma=sigma)
    x = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    u, gr, _ = pl.pointwise(sc, params, x, with_grad=True)
    torch.cuda.synchronize()
    uo, go, _ = orc.pointwise(orc.Scene(scene), g, f, orc.walk_params(1e-3, W, 99, sigma=sigma), pts)
    oku = per_walk_match(u.cpu().numpy(), uo, 1e-9)
    okg = per_walk_match(to_np_aos(gr), go, 1e-8).all(axis=1)
    say(f"  points {pts.shape[0]}: u {oku.mean():.4f} grad {okg.mean():.4f}")
    assert oku.mean() >= 0.99 and okg.mean() >= 0.99


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_source_fp32_statistical(orc, dim):
    _bvc, pl = lib()
    scene, g, f, _ = _case(dim, SIG)
    say(f"screened source fp32 dim={dim}")
    sc = pl.Scene(scene)
    gd, fd = pl.DeviceField(g), pl.DeviceField(f)
    pts = _interior(orc, scene, 48, 6)
    W = 512
    x = torch.from_numpy(np.ascontiguousarray(pts.T)).to("cuda", torch.float32)
    # per-walk samples from the device (pointwise walks, FP32)
    params = pl.walk_params(1e-3, W, 131, gd, fd, "f32", sigma=SIG)
    n = pts.shape[0]
    Uw = torch.empty(n * W, dtype=torch.float32, device="cuda")
    work = torch.empty(_bvc.bvc_pointwise_workspace_bytes(dim, n, W, _bvc.F32, False), dtype=torch.uint8,
                       device="cuda")
    u = torch.empty(n, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    _bvc.bvc_pointwise_wos(sc.h, params, n, x, Uw, None, work, u, None, cnt)
    torch.cuda.synchronize()
    A = Uw.double().cpu().numpy().reshape(n, W)
    # the oracle's means and standard errors on independent streams
    ob = []
    for bt in range(8):
        uo, _, _ = orc.pointwise(orc.Scene(scene), g, f, orc.walk_params(1e-3, W // 8, 2131 + bt, sigma=SIG), pts,
                                 with_grad=False)
        ob.append(uo)
    ob = np.array(ob)
    se = np.sqrt(A.var(1, ddof=1) / W + ob.var(0, ddof=1) / 8) + 1e-12
    ok, msg = z_ok(np.abs(A.mean(1) - ob.mean(0)) / se)
    say(f"  {msg}")
    assert ok, msg


def test_screened_step_with_source_against_closed_form():
    _bvc, pl = lib()
    dim, sigma = 2, 4.0
    scene, g, f, b = _case(dim, sigma)
    lo, hi = scene.bbox
    eps = 1e-3 * scene.diagonal
    prob = wl.Problem("circle_screened_source", scene, g, f, 4096, 128, eps, 5 * eps, 4096,
                      wl.grid2d(96, lo, hi), g, sides=1, precision="f32", seed_walks=71, seed_cache=72,
                      seed_sources=73, sigma=sigma)
    prep = pl.Prepared(prob)
    sol = pl.solve(prep, batch=2, with_grad=False)
    torch.cuda.synchronize()
    idx = prep.idx_int[: prep.n_int].cpu().numpy()
    d = prep.dist[idx].cpu().numpy()
    u = sol.u_int[: prep.n_int].double().cpu().numpy()
    truth = wl.field_value(g, prob.eval_x[idx])
    far = d >= 0.1
    rmse = float(np.sqrt(np.mean((u[far] - truth[far]) ** 2)))
    rms = float(np.sqrt(np.mean(truth ** 2)))
    ub = sol.u_band[: prep.n_band].double().cpu().numpy()
    tb = wl.field_value(g, prob.eval_x[prep.idx_band[: prep.n_band].cpu().numpy()])
    rb = float(np.sqrt(np.mean((ub - tb) ** 2)))
    say(f"  gathered {far.sum()} at d >= 0.1: rmse {rmse:.4g} (rms u {rms:.3g}); band {ub.size}: rmse {rb:.4g}")
    assert rmse <= 0.02 * rms and rb <= 0.02 * rms
