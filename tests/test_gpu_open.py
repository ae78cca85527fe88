"""GPU parity of open (unbounded) 3D domains (Appendix B): walks in the
exterior of a closed mesh that escape to infinity (u = 0) or re-enter on a
sphere enclosing the mesh, against the FP64 oracle through the C-ABI
(marked gpu).

- FP64 cache walks walk by walk on the oracle's Philox streams: U and D
  (at least 99.9% within 1e-9), the same walks escape (NaN exit records),
  exit points and step counts agree.
- FP64 pointwise walks from points near and far from the solid (means of u
  and grad u per point).
- FP32 cache walks against the FP64 oracle walks on the same streams
  (z-test of the mean difference).
- The whole step outside the displaced sphere recovers u = 1/|x - q|.
- Basis means (adjoint and multi-field paths): escaped walks count as u = 0;
  device on the oracle's records matches the oracle, and E theta, F theta
  reproduce the walks of g = sum theta_m phi_m.
- Refusals: a sphere that leaves out a vertex, a source, screening, 2D
  scenes, the batch and walk-on-stars calls.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, oracle_cache, per_walk_match, to_np_aos

pytestmark = pytest.mark.gpu

Q = (0.1, -0.05, 0.07)


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return lib()


def _case(pl):
    scene = wl.exterior_of(wl.displaced_icosphere(3, 31))
    return scene, pl.Scene(scene), wl.point_source(1.0, Q), wl.enclosing_sphere(scene)


def test_open_walks_fp64_walk_by_walk(B, orc):
    _bvc, pl = B
    say("open-domain walks fp64")
    scene, sc, g, sph = _case(pl)
    gd = pl.DeviceField(g)
    eps, l, W, seed = 1e-3, 2e-2, 8, 91
    cache = pl.sample_cache(sc, 900, l, 1, 5, 0)
    wp = pl.walk_params(eps, W, seed, gd, None, "f64", open_sphere=sph)
    U, D, rec, counters = pl.cache_walks(sc, cache, wp, "f64", records=True)
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    ref = orc.cache_walks(osc, g, None, orc.walk_params(eps, W, seed, open_sphere=sph),
                          oracle_cache(osc.sample_cache(900, l, 1, 5, 0), cache), records=True)
    n = cache.n * W
    okU = per_walk_match(U.cpu().numpy()[:n], ref["U"])
    okD = per_walk_match(D.cpu().numpy()[:n], ref["D"])
    ex_g, ex_o = to_np_aos(rec["exit"], n), ref["exit"]
    esc_g, esc_o = np.isnan(ex_g[:, 0]), np.isnan(ex_o[:, 0])
    both = ~esc_g & ~esc_o
    okX = np.all(np.abs(ex_g[both] - ex_o[both]) <= 1e-9, axis=1)
    okS = rec["steps"].cpu().numpy()[:n] == ref["steps"]
    say(f"  cache walks {n}: U {okU.mean():.5f} D {okD.mean():.5f} escaped {esc_o.mean():.4f} "
        f"same escapes {(esc_g == esc_o).mean():.5f} exits {okX.mean():.5f} steps {okS.mean():.5f}")
    assert esc_o.sum() >= 20
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999
    assert (esc_g == esc_o).mean() >= 0.999 and okX.mean() >= 0.999 and okS.mean() >= 0.999
    # pointwise walks from points near and far from the solid
    rng = np.random.default_rng(4)
    v = rng.normal(0, 1, (160, 3))
    x = v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.9, 5.0, 160)[:, None]
    x = x[osc.inside(x) != 0]
    Wp = 16
    wpp = pl.walk_params(eps, Wp, seed, gd, None, "f64", open_sphere=sph)
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")
    u, gr, cnt = pl.pointwise(sc, wpp, xd, True)
    torch.cuda.synchronize()
    uo, go, _ = orc.pointwise(osc, g, None, orc.walk_params(eps, Wp, seed, open_sphere=sph), x, with_grad=True)
    oku = per_walk_match(u.cpu().numpy()[: x.shape[0]], uo)
    okg = np.all(np.abs(to_np_aos(gr, x.shape[0]) - go) <= 1e-9 * (np.abs(go) + np.sqrt(np.mean(go**2))), axis=1)
    say(f"  pointwise means {x.shape[0]}: u {oku.mean():.4f} grad {okg.mean():.4f}")
    assert oku.mean() >= 0.99 and okg.mean() >= 0.99


def test_open_walks_fp32_statistical(B, orc):
    _bvc, pl = B
    say("open-domain walks fp32")
    scene, sc, g, sph = _case(pl)
    gd = pl.DeviceField(g)
    eps, l, W, seed = 1e-3, 2e-2, 64, 92
    cache = pl.sample_cache(sc, 300, l, 1, 6, 0)
    wp = pl.walk_params(eps, W, seed, gd, None, "f32", open_sphere=sph)
    U, D, rec, counters = pl.cache_walks(sc, cache, wp, "f32")
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    ref = orc.cache_walks(osc, g, None, orc.walk_params(eps, W, seed, open_sphere=sph),
                          oracle_cache(osc.sample_cache(300, l, 1, 6, 0), cache))
    n = cache.n * W
    for name in ("U", "D"):
        A = (U if name == "U" else D).double().cpu().numpy()[:n]
        diff = A - ref[name]
        assert np.all(np.isfinite(A))
        z = diff.mean() / (diff.std(ddof=1) / np.sqrt(n) + 1e-300)
        close = per_walk_match(A, ref[name], 1e-3).mean()
        say(f"  {name}: z {z:.2f}, within 1e-3 {close:.4f}")
        assert abs(z) < 5 and close > 0.95


def test_pipeline_open_sphere(B):
    """The whole step (FP32) outside the displaced sphere recovers the decaying
    potential u = 1/|x - q| at gathered and band points."""
    _bvc, pl = B
    say("pipeline open sphere")
    prob = wl.problem_c3_open(n_eval_box=20000)
    prep = pl.Prepared(prob, dtype="f32")
    sol = pl.solve(prep, with_grad=True)
    torch.cuda.synchronize()
    idx = prep.idx_int[: prep.n_int].cpu().numpy()
    pts = prob.eval_x[idx]
    truth = wl.field_value(prob.truth, pts)
    u = sol.u_int[: prep.n_int].double().cpu().numpy()
    d = prep.dist[prep.idx_int[: prep.n_int].long()].cpu().numpy()
    far = d > 0.05
    rms = np.sqrt(np.mean(truth**2))
    err = np.sqrt(np.mean((u[far] - truth[far]) ** 2))
    say(f"  gathered {prep.n_int}: rmse {err:.4g} (mean {np.mean(u[far] - truth[far]):.3g}) vs rms {rms:.4g}")
    assert prep.n_int > 10000 and err < 0.02 * rms
    r = pts - np.array(Q)[None]
    gt = -r / np.linalg.norm(r, axis=1, keepdims=True) ** 3
    gerr = np.sqrt(np.sum((to_np_aos(sol.g_int, prep.n_int) - gt) ** 2, 1))
    gn = np.sqrt(np.mean(np.sum(gt**2, 1)))
    m = d > 0.2
    say(f"  grad rmse (d > 0.2): {np.sqrt(np.mean(gerr[m] ** 2)) / gn:.4f} of rms, {m.sum()} points")
    assert np.sqrt(np.mean(gerr[m] ** 2)) < 0.05 * gn
    nb = prep.n_band
    if nb:
        ib = prep.idx_band[:nb].cpu().numpy()
        tb = wl.field_value(prob.truth, prob.eval_x[ib])
        ub = sol.u_band[:nb].double().cpu().numpy()
        say(f"  band {nb}: rmse {np.sqrt(np.mean((ub - tb) ** 2)):.4g}")
        assert np.sqrt(np.mean((ub - tb) ** 2)) < 0.02 * np.sqrt(np.mean(tb**2))


def test_open_domain_refusals(B):
    _bvc, pl = B
    say("open-domain refusals")
    scene, sc, g, (c, r) = _case(pl)
    gd = pl.DeviceField(g)
    cache = pl.sample_cache(sc, 64, 2e-2, 1, 5, 0)

    def walks(**kw):
        wp = pl.walk_params(1e-3, 2, 1, gd, kw.pop("f", None), "f32", **kw)
        pl.cache_walks(sc, cache, wp, "f32")

    with pytest.raises(RuntimeError, match="enclose"):
        walks(open_sphere=(c, 0.5 * r))
    with pytest.raises(RuntimeError, match="Laplace"):
        walks(open_sphere=(c, r), sigma=1.0)
    with pytest.raises(RuntimeError, match="Laplace"):
        walks(open_sphere=(c, r), f=pl.DeviceField(wl.Field(1, [], [1.0])))
    with pytest.raises(RuntimeError, match="positive"):
        walks(open_sphere=(c, -1.0))
    sc2 = pl.Scene(wl.circle_polygon(64))
    c2 = pl.sample_cache(sc2, 64, 2e-2, 1, 5, 0)
    wp = pl.walk_params(1e-3, 2, 1, pl.DeviceField(wl.point_source(1.0, (0.1, 0.0))), None, "f32",
                        open_sphere=((0.0, 0.0, 0.0), 2.0))
    with pytest.raises(RuntimeError, match="3D"):
        pl.cache_walks(sc2, c2, wp, "f32")
    torch.cuda.synchronize()


@pytest.mark.parametrize("lmax", [8, 10])
def test_open_basis_means_fp64(B, orc, lmax):
    """Basis means of the adjoint and multi-field paths on open-domain walks:
    an escaped walk contributes 0 to every basis mean (u = 0 at infinity) and
    its control-variate term to F.  The device kernel on the oracle's records
    matches the oracle; E theta and F theta reproduce the walks of
    g = sum theta_m phi_m on the same streams (the escapes do not depend on g)."""
    _bvc, pl = B
    say(f"open-domain basis means lmax {lmax}")
    scene, sc, _, sph = _case(pl)
    nb = (lmax + 1) ** 2
    theta = np.random.default_rng(8).normal(0, 1, nb)
    basis, g = wl.solid_harmonics_3d(np.zeros(nb), lmax), wl.solid_harmonics_3d(theta, lmax)
    eps, l, W = 1e-3, 2e-2, 8
    cache = pl.sample_cache(sc, 500, l, 1, 7, 0)
    gd = pl.DeviceField(g)  # the walk parameters hold only its device pointer
    U, D, rec, _ = pl.cache_walks(sc, cache, pl.walk_params(eps, W, 17, gd, None, "f64", open_sphere=sph), "f64",
                                  records=True)
    bd = pl.DeviceField(basis)
    E = torch.empty(cache.n, nb, dtype=torch.float64, device="cuda")
    F = torch.empty_like(E)
    _bvc.bvc_basis_means(bd.c(), 3, cache.n, W, _bvc.F64, rec["exit"], rec["w1"], cache.xbar, 1, E, F)
    osc = orc.Scene(scene)
    cn = oracle_cache(osc.sample_cache(500, l, 1, 7, 0), cache)
    ref = orc.cache_walks(osc, g, None, orc.walk_params(eps, W, 17, open_sphere=sph), cn, records=True)
    assert np.isnan(ref["exit"][:, 0]).sum() >= 5
    Eo, Fo = orc.basis_means(basis, 3, ref["exit"], ref["w1"], cn["xbar"], W)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.T if a.ndim == 2 else a)).to("cuda")
    E2, F2 = torch.empty_like(E), torch.empty_like(F)
    _bvc.bvc_basis_means(bd.c(), 3, cache.n, W, _bvc.F64, dev(ref["exit"]), dev(ref["w1"]), dev(cn["xbar"]), 1,
                         E2, F2)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(E.cpu().numpy())) and np.all(np.isfinite(F.cpu().numpy()))
    assert np.allclose(E2.cpu().numpy(), Eo, rtol=1e-10, atol=1e-11)
    assert np.allclose(F2.cpu().numpy(), Fo, rtol=1e-9, atol=1e-9)
    Um = U.cpu().numpy()[: cache.n * W].reshape(-1, W).mean(1)
    Dm = D.cpu().numpy()[: cache.n * W].reshape(-1, W).mean(1)
    s_u, s_d = np.sqrt(np.mean(Um**2)), np.sqrt(np.mean(Dm**2))
    say(f"  escaped {np.isnan(ref['exit'][:, 0]).mean():.4f}; |E theta - U| {np.abs(E.cpu().numpy() @ theta - Um).max():.3g}")
    assert np.allclose(E.cpu().numpy() @ theta, Um, rtol=0, atol=1e-9 * s_u)
    assert np.allclose(F.cpu().numpy() @ theta, Dm, rtol=0, atol=1e-9 * s_d)
