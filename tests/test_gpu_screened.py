"""GPU parity of the screened Poisson path (Eq. 1 with sigma > 0, 2D and 3D;
Appendix A.2) against the FP64 oracle, through the C-ABI (marked gpu).

- Screened gather (u, grad u, sources): FP64 to 1e-11 of the sum of |terms|,
  FP32 to the per-term FP32 bound of the plain gather test.
- Screened walks, FP64: cache walks (U, D) and pointwise walks (U, grad)
  walk by walk on the oracle's Philox streams (at least 99.9% within 1e-9);
  FP32: walk means against the FP64 walks on the same streams (z-test).
- The pipeline on the screened sphere and star problems recovers exp(a.x).
- Unsupported combinations (near field or clamp with screening, the
  clamping correction) are refused with an error; a walk source with
  screening is built and tested in test_gpu_sources.py.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, oracle_cache, per_walk_match, to_np_aos

pytestmark = pytest.mark.gpu

SIGMA = 4.0


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return lib()


def _plane(dim=3):
    a = np.array([1.0, 0.5, -0.7])[:dim]
    return wl.exp_plane(1.0, a / np.linalg.norm(a) * np.sqrt(SIGMA))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_screened_gather_matches_oracle(B, orc, dtype, dim):
    _bvc, pl = B
    say(f"screened gather {dim}d {dtype}")
    rng = np.random.default_rng(21 + dim)
    N, M, K = 1300, 700, 1537
    th = rng.normal(0, 1, (N, dim))
    cy = th / np.linalg.norm(th, axis=1, keepdims=True) * 1.01
    cn = cy / np.linalg.norm(cy, axis=1, keepdims=True)
    a, b = rng.normal(0, 1, N) / N, rng.normal(0, 1, N) / N
    sy, sw = rng.uniform(-0.7, 0.7, (M, dim)), rng.normal(0, 1, M) / M
    v = rng.normal(0, 1, (K, dim))
    ex = v / np.linalg.norm(v, axis=1, keepdims=True) * (0.95 * rng.random(K) ** (1 / dim))[:, None]
    T = torch.float64 if dtype == "f64" else torch.float32
    code = _bvc.F64 if dtype == "f64" else _bvc.F32
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x.T if x.ndim == 2 else x)).to("cuda", T)
    cache = dict(n=N, dtype=code, x=dev(cy), nrm=dev(cn), a=dev(a), b=dev(b))
    src = dict(n=M, dtype=code, y=dev(sy), s=dev(sw))
    u = torch.empty(K, dtype=T, device="cuda")
    g = torch.empty(dim, K, dtype=T, device="cuda")
    u2 = torch.empty(K, dtype=T, device="cuda")
    _bvc.bvc_gather_grad(dim, cache, src, K, dev(ex), u, g, sigma=SIGMA)
    _bvc.bvc_gather_u(dim, cache, src, K, dev(ex), u2, sigma=SIGMA)
    torch.cuda.synchronize()
    r64 = lambda t: t.double().cpu().numpy()
    cy_r, cn_r, a_r, b_r = to_np_aos(cache["x"]), to_np_aos(cache["nrm"]), r64(cache["a"]), r64(cache["b"])
    ex_r, sy_r, sw_r = to_np_aos(dev(ex)), to_np_aos(src["y"]), r64(src["s"])
    uo, go, cond = orc.gather_sigma(dim, SIGMA, ex_r, cy_r, cn_r, a_r, b_r, sy_r, sw_r, with_grad=True,
                                    with_cond=True)
    up = orc.gather(dim, ex_r, cy_r, cn_r, a_r, b_r, sy_r, sw_r, with_grad=False)
    assert np.mean(np.abs(uo - up)) > 1e-3 * np.mean(cond)  # screening changes the result
    ug, gg = u.double().cpu().numpy(), to_np_aos(g)
    if dtype == "f64":
        assert np.all(np.abs(ug - uo) <= 1e-11 * cond)
        assert np.all(np.abs(u2.cpu().numpy() - uo) <= 1e-11 * cond)
        assert np.all(np.abs(gg - go).max(1) <= 1e-10 * (np.abs(go).max(1) + cond))
    else:
        uu = 2.0**-24
        zall = np.concatenate([cy_r, sy_r])
        rmin = np.min(np.linalg.norm(ex_r[:, None, :] - zall[None], axis=2), axis=1)
        zmax = np.linalg.norm(zall, axis=1).max()
        tol = uu * cond * (300 + 4 * (np.linalg.norm(ex_r, axis=1) + zmax) / rmin) + uu * np.abs(uo)
        assert np.all(np.abs(ug - uo) <= tol), np.max(np.abs(ug - uo) / tol)
        if dim == 3:
            gsum = (4 * np.abs(a_r).sum() / rmin**3 + (np.abs(b_r).sum() + np.abs(sw_r).sum()) / rmin**2) / (4 * np.pi)
        else:
            lg = np.abs(np.log(np.sqrt(SIGMA) * rmin)) + 1
            gsum = (3 * np.abs(a_r).sum() / rmin**2 + SIGMA * lg * np.abs(a_r).sum() / rmin
                    + (np.abs(b_r).sum() + np.abs(sw_r).sum()) / rmin) / (2 * np.pi)
        gtol = uu * gsum * (300 + 4 * (np.linalg.norm(ex_r, axis=1) + zmax) / rmin) + uu * np.abs(go).max(1)
        assert np.all(np.abs(gg - go).max(1) <= gtol)


def _sphere_case(pl, dim=3):
    scene = wl.displaced_icosphere(3, 31) if dim == 3 else wl.star_polygon(512, 11, jitter="radial", sigma=0.01)
    sc = pl.Scene(scene)
    g = _plane(dim)
    return scene, sc, g


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_walks_fp64_walk_by_walk(B, orc, dim):
    _bvc, pl = B
    say(f"screened walks fp64 {dim}d")
    scene, sc, g = _sphere_case(pl, dim)
    gd = pl.DeviceField(g)
    eps, l, W, seed = 4e-3, 2e-2, 8, 77
    cache = pl.sample_cache(sc, 600, l, 1, 5, 0)
    wp = pl.walk_params(eps, W, seed, gd, None, "f64", sigma=SIGMA)
    U, D, rec, counters = pl.cache_walks(sc, cache, wp, "f64")
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    P = orc.walk_params(eps, W, seed, sigma=SIGMA)
    ref = orc.cache_walks(osc, g, None, P, oracle_cache(osc.sample_cache(600, l, 1, 5, 0), cache))
    n = cache.n * W
    okU = per_walk_match(U.cpu().numpy()[:n], ref["U"])
    okD = per_walk_match(D.cpu().numpy()[:n], ref["D"])
    say(f"  cache walks {n}: U {okU.mean():.5f} D {okD.mean():.5f}")
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999
    # pointwise walks (u and grad), some starting inside the epsilon shell
    rng = np.random.default_rng(3)
    v = rng.normal(0, 1, (150, dim))
    x = v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.2, 0.97, 150)[:, None]
    d0, _, _ = osc.closest(x)
    x = x[osc.inside(x) != 0]
    Wp = 16
    wpp = pl.walk_params(eps, Wp, seed, gd, None, "f64", sigma=SIGMA)
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda")
    u, gr, cnt = pl.pointwise(sc, wpp, xd, True)
    torch.cuda.synchronize()
    uo, go, _ = orc.pointwise(osc, g, None, orc.walk_params(eps, Wp, seed, sigma=SIGMA), x, with_grad=True)
    oku = per_walk_match(u.cpu().numpy()[: x.shape[0]], uo)
    okg = np.all(np.abs(to_np_aos(gr, x.shape[0]) - go) <= 1e-9 * (np.abs(go) + np.sqrt(np.mean(go**2))), axis=1)
    say(f"  pointwise means {x.shape[0]}: u {oku.mean():.4f} grad {okg.mean():.4f}")
    assert oku.mean() >= 0.99 and okg.mean() >= 0.99


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_walks_fp32_statistical(B, orc, dim):
    _bvc, pl = B
    say(f"screened walks fp32 {dim}d")
    scene, sc, g = _sphere_case(pl, dim)
    gd = pl.DeviceField(g)
    eps, l, W, seed = 4e-3, 2e-2, 64, 78
    cache = pl.sample_cache(sc, 150, l, 1, 6, 0)
    wp = pl.walk_params(eps, W, seed, gd, None, "f32", sigma=SIGMA)
    U, D, rec, counters = pl.cache_walks(sc, cache, wp, "f32")
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    ref = orc.cache_walks(osc, g, None, orc.walk_params(eps, W, seed, sigma=SIGMA),
                          oracle_cache(osc.sample_cache(150, l, 1, 6, 0), cache))
    n = cache.n
    for name in ("U", "D"):
        A = (U if name == "U" else D).double().cpu().numpy()[: n * W].reshape(n, W)
        Bo = ref[name].reshape(n, W)
        se = np.sqrt(A.var(1) / W + Bo.var(1) / W) + 1e-12
        z = (A.mean(1) - Bo.mean(1)) / se
        say(f"  {name}: max |z| {np.abs(z).max():.2f}")
        assert np.all(np.abs(z) < 5)
        assert abs(z.mean() * np.sqrt(n)) < 5


def test_pipeline_screened_sphere(B):
    """The whole step on the screened sphere problem (FP32) recovers the plane
    wave exp(a.x) at interior points to a few percent of its RMS."""
    _bvc, pl = B
    say("pipeline screened sphere")
    prob = wl.problem_c3_screened(n_eval_box=20000)
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
    bias = np.mean(u[far] - truth[far])
    say(f"  interior {prep.n_int}: rmse {err:.4g} (mean {bias:.3g}) vs rms {rms:.4g}")
    assert err < 0.02 * rms
    gt = np.array(prob.truth.param[1:4])[None] * truth[:, None]
    gerr = np.sqrt(np.sum((to_np_aos(sol.g_int, prep.n_int) - gt) ** 2, 1))
    gn = np.sqrt(np.mean(np.sum(gt**2, 1)))
    for lo in (0.05, 0.1, 0.2, 0.3):
        m = d > lo
        say(f"  grad rmse (d > {lo}): {np.sqrt(np.mean(gerr[m] ** 2)) / gn:.4f} of rms, {m.sum()} points")
    m = d > 0.2
    assert np.sqrt(np.mean(gerr[m] ** 2)) < 0.04 * gn


def test_pipeline_screened_star(B):
    """The whole 2D step on the screened star problem (FP32) recovers the
    plane wave exp(a.x) at interior points to a few percent of its RMS."""
    _bvc, pl = B
    say("pipeline screened star")
    prob = wl.problem_c2_screened(grid=256)
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
    say(f"  interior {prep.n_int}: rmse {err:.4g} vs rms {rms:.4g}")
    assert err < 0.02 * rms
    gt = np.array(prob.truth.param[1:3])[None] * truth[:, None]
    gerr = np.sqrt(np.sum((to_np_aos(sol.g_int, prep.n_int) - gt) ** 2, 1))
    gn = np.sqrt(np.mean(np.sum(gt**2, 1)))
    m = d > 0.2
    say(f"  grad rmse (d > 0.2): {np.sqrt(np.mean(gerr[m] ** 2)) / gn:.4f} of rms, {m.sum()} points")
    assert np.sqrt(np.mean(gerr[m] ** 2)) < 0.04 * gn
    ub = sol.u_band[: prep.n_band].double().cpu().numpy()
    tb = wl.field_value(prob.truth, prob.eval_x[prep.idx_band[: prep.n_band].cpu().numpy()])
    assert np.sqrt(np.mean((ub - tb) ** 2)) < 0.02 * rms


def test_screened_unsupported_combinations(B):
    _bvc, pl = B
    say("screened unsupported combinations")
    scene, sc, g = _sphere_case(pl)
    gd = pl.DeviceField(g)
    # (a source with screening is built: tests/test_gpu_sources.py)
    T = torch.float64
    cv = dict(n=4, dtype=_bvc.F64, x=torch.ones(3, 4, dtype=T, device="cuda"),
              nrm=torch.ones(3, 4, dtype=T, device="cuda"), a=torch.ones(4, dtype=T, device="cuda"),
              b=torch.ones(4, dtype=T, device="cuda"))
    u = torch.empty(4, dtype=T, device="cuda")
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_gather_u(3, cv, None, 4, torch.zeros(3, 4, dtype=T, device="cuda"), u, sigma=1.0, clamp=2.0)
    wp = pl.walk_params(4e-3, 1, 1, gd, None, "f64", sigma=1.0)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(6, dtype=torch.int64, device="cuda")
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_clamp_correction(sc.h, wp, _bvc.clamp_params(0.02, 1, 5.0, 4, 2), 4,
                                  torch.zeros(3, 4, dtype=T, device="cuda"), None, None, u, ws, cnt)
