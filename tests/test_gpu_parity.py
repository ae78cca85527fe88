"""GPU parity of the HIP path against the FP64 oracle (marked gpu).

Every case runs the library through its C-ABI (ctypes binding) on cuda:0 and
compares element by element with the oracle on the same inputs:
  - integer decisions (accept flags, classification, step counts): exact;
  - FP64 walks: per walk |gpu - oracle| <= 1e-9 max(|oracle|, RMS) for at
    least 99.9% of walks (identical Philox streams; the rest may differ when
    an ulp-level difference flips a termination or closest-primitive
    decision);
  - FP64 gather / adjoint / basis means: 1e-10 relative to the sum of |terms|;
  - FP32 gather: 64 u (16 + 4 (|x| + |z|)/r) per term summed (the FP32
    rounding of the difference x - z and of the kernel evaluation).
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import abs_terms as _abs_terms
from gpu_helpers import c2_like_fields, lib, oracle_cache, per_walk_match, small_star, to_np_aos, z_ok

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return lib()


def _dev(v):
    """A host array on the device in the library's [dim][n] layout."""
    return torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", torch.float64)


def _prep(pl, scene, g, f=None):
    sc = pl.Scene(scene)
    return sc, pl.DeviceField(g), (pl.DeviceField(f) if f is not None else None)


CASES = {
    "c1": lambda: (wl.circle_polygon(128), wl.harmonic_2d(3, 1.0, 1.0), None, 1e-3, 5e-3, 1, 1300, 16),
    "star_poisson": lambda: (small_star(), *c2_like_fields(), 3e-3, 1.5e-2, 2, 2500, 8),
    "sphere_sh": lambda: (wl.displaced_icosphere(3, 31), wl.solid_harmonics_3d(
        np.random.default_rng(1).normal(0, 1, 81), 8), None, 4e-3, 2e-2, 1, 600, 8),
}


@pytest.mark.parametrize("case", list(CASES))
def test_sampler_matches_oracle(B, orc, case):
    _bvc, pl = B
    scene, g, f, eps, l, sides, n, W = CASES[case]()
    say(f"sampler {case} n={n}")
    sc, _, _ = _prep(pl, scene, g)
    d = scene.dim
    x = torch.empty(d, n, dtype=torch.float64, device="cuda")
    nrm, xbar = torch.empty_like(x), torch.empty_like(x)
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    R0 = torch.empty_like(w)
    acc = torch.empty(n, dtype=torch.int32, device="cuda")
    _bvc.bvc_sample_cache(sc.h, n, l, sides, 123, 5, x, nrm, w, xbar, R0, acc)
    torch.cuda.synchronize()
    ref = orc.Scene(scene).sample_cache(n, l, sides, 123, 5)
    got_acc = acc.cpu().numpy().astype(bool)
    assert np.array_equal(got_acc, ref["accept"])
    assert np.allclose(to_np_aos(x), ref["x"], rtol=0, atol=1e-13)
    assert np.allclose(to_np_aos(xbar), ref["xbar"], rtol=0, atol=1e-13)
    assert np.allclose(R0.cpu().numpy(), ref["R0"], rtol=1e-12, atol=1e-15)
    assert np.allclose(w.cpu().numpy(), ref["w"], rtol=1e-14)
    m = got_acc
    assert np.allclose(to_np_aos(nrm)[m], ref["n"][m], atol=1e-9)
    # compaction keeps the accepted candidates in order
    cache = pl.sample_cache(sc, n, l, sides, 123, 5)
    assert cache.n == int(m.sum())
    assert np.allclose(to_np_aos(cache.x, cache.n), ref["x"][m], rtol=0, atol=1e-13)


@pytest.mark.parametrize("case", list(CASES))
def test_classify_matches_oracle(B, orc, case):
    _bvc, pl = B
    scene, g, f, eps, l, sides, n, W = CASES[case]()
    say(f"classify {case}")
    sc, _, _ = _prep(pl, scene, g)
    lo, hi = scene.bbox
    pts = wl.uniform_box(3000, lo - 0.05, hi + 0.05, 9)
    cls, dist = pl.classify(sc, torch.from_numpy(np.ascontiguousarray(pts.T)).cuda(), l)
    ref = orc.Scene(scene).classify(pts, l)
    assert np.array_equal(cls.cpu().numpy(), ref)
    d_ref, _, _ = orc.Scene(scene).closest(pts)
    assert np.allclose(dist.cpu().numpy(), d_ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("case", list(CASES))
def test_cache_walks_fp64_per_walk(B, orc, case):
    _bvc, pl = B
    scene, g, f, eps, l, sides, n, W = CASES[case]()
    say(f"cache walks fp64 {case} n={n} W={W}")
    sc, gd, fd = _prep(pl, scene, g, f)
    cache = pl.sample_cache(sc, n, l, sides, 77, 0)
    params = pl.walk_params(eps, W, 4242, gd, fd, "f64")
    U, D, rec, counters = pl.cache_walks(sc, cache, params, "f64", records=True)
    torch.cuda.synchronize()
    os_ = orc.Scene(scene)
    cn = oracle_cache(os_.sample_cache(n, l, sides, 77, 0), cache)
    P = orc.walk_params(eps, W, 4242)
    ref = orc.cache_walks(os_, g, f, P, cn, records=True)
    Ug = U.cpu().numpy()[: cache.n * W]
    Dg = D.cpu().numpy()[: cache.n * W]
    okU = per_walk_match(Ug, ref["U"])
    okD = per_walk_match(Dg, ref["D"])
    steps = rec["steps"].cpu().numpy()[: cache.n * W]
    say(f"  walks={Ug.size} U-match={okU.mean():.5f} D-match={okD.mean():.5f} steps={steps.sum()}")
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999
    assert np.mean(steps == ref["steps"]) >= 0.999
    c = counters.cpu().numpy()
    assert c[3] == Ug.size and c[1] == steps.sum()
    # exit records
    ex = to_np_aos(rec["exit"], cache.n * W)
    assert np.mean(np.all(np.abs(ex - ref["exit"]) < 1e-9, axis=1)) >= 0.999
    assert np.mean(per_walk_match(rec["w1"].cpu().numpy()[: cache.n * W], ref["w1"])) >= 0.999
    # reduction in FP64: the device kernel on the oracle's walks
    uhat, dudn, a, b = pl.reduce_walks(cache, W, _dev(ref["U"]), _dev(ref["D"]), "f64")
    uh_ref, dh_ref = orc.reduce(ref["U"], ref["D"], W)
    assert np.allclose(uhat.cpu().numpy()[: cache.n], uh_ref, rtol=1e-12, atol=1e-14)
    assert np.allclose(dudn.cpu().numpy()[: cache.n], dh_ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(a.cpu().numpy()[: cache.n], uh_ref * cn["w"], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("case", ["c1", "star_poisson", "sphere_sh"])
def test_pointwise_fp64_per_walk(B, orc, case):
    _bvc, pl = B
    scene, g, f, eps, l, sides, n, W = CASES[case]()
    say(f"pointwise fp64 {case}")
    sc, gd, fd = _prep(pl, scene, g, f)
    lo, hi = scene.bbox
    pts = wl.uniform_box(400, lo * 0.7, hi * 0.7, 3)
    os_ = orc.Scene(scene)
    pts = pts[os_.inside(pts) != 0][:200]
    x = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    Wp = 16
    params = pl.walk_params(eps, Wp, 99, gd, fd, "f64")
    u, gr, cnt = pl.pointwise(sc, params, x, with_grad=True)
    torch.cuda.synchronize()
    uo, go, tot = orc.pointwise(os_, g, f, orc.walk_params(eps, Wp, 99), pts)
    okp = per_walk_match(u.cpu().numpy(), uo, 1e-9)
    assert okp.mean() >= 0.99
    assert np.mean(per_walk_match(to_np_aos(gr), go, 1e-8).all(axis=1)) >= 0.99
    assert abs(int(cnt.cpu().numpy()[1]) - tot) <= 0.001 * tot + 2


def _gather_case(dim, dtype):
    rng = np.random.default_rng(dim + (10 if dtype == "f32" else 0))
    N, M, K = 1300, 700, 1537  # several tiles and ragged tails
    th = rng.normal(0, 1, (N, dim))
    cy = th / np.linalg.norm(th, axis=1, keepdims=True) * 1.01
    cn = cy / np.linalg.norm(cy, axis=1, keepdims=True)
    a = rng.normal(0, 1, N) / N
    b = rng.normal(0, 1, N) / N
    r = 0.95 * rng.random(K) ** (1.0 / dim)
    d = rng.normal(0, 1, (K, dim))
    ex = d / np.linalg.norm(d, axis=1, keepdims=True) * r[:, None]
    sy = rng.uniform(-0.7, 0.7, (M, dim))
    sw = rng.normal(0, 1, M) / M
    return ex, cy, cn, a, b, sy, sw


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_matches_oracle(B, orc, dim, dtype):
    _bvc, pl = B
    say(f"gather dim={dim} {dtype}")
    ex, cy, cn, a, b, sy, sw = _gather_case(dim, dtype)
    T = torch.float64 if dtype == "f64" else torch.float32
    code = _bvc.F64 if dtype == "f64" else _bvc.F32

    def dev(v, rows=True):
        return torch.from_numpy(np.ascontiguousarray(v.T if (rows and v.ndim == 2) else v)).to("cuda", T)

    cache = dict(n=cy.shape[0], dtype=code, x=dev(cy), nrm=dev(cn), a=dev(a), b=dev(b))
    src = dict(n=sy.shape[0], dtype=code, y=dev(sy), s=dev(sw))
    K = ex.shape[0]
    u = torch.empty(K, dtype=T, device="cuda")
    g = torch.empty(dim, K, dtype=T, device="cuda")
    _bvc.bvc_gather_grad(dim, cache, src, K, dev(ex), u, g)
    u2 = torch.empty(K, dtype=T, device="cuda")
    _bvc.bvc_gather_u(dim, cache, src, K, dev(ex), u2)
    torch.cuda.synchronize()
    # inputs as the device holds them (FP32 rounding included)
    r64 = lambda t: t.double().cpu().numpy()
    cy_r, cn_r, a_r, b_r = (to_np_aos(cache["x"]), to_np_aos(cache["nrm"]), r64(cache["a"]), r64(cache["b"]))
    ex_r, sy_r, sw_r = to_np_aos(dev(ex)), to_np_aos(src["y"]), r64(src["s"])
    uo, go, cond = orc.gather(dim, ex_r, cy_r, cn_r, a_r, b_r, sy_r, sw_r, with_grad=True, with_cond=True)
    ug, gg = u.double().cpu().numpy(), to_np_aos(g)
    if dtype == "f64":
        tol = 1e-11 * cond + 1e-300
        assert np.all(np.abs(ug - uo) <= tol)
        assert np.all(np.abs(u2.cpu().numpy() - uo) <= tol)
        gs = np.abs(go).max(1) + cond
        assert np.all(np.abs(gg - go).max(1) <= 1e-10 * gs)
    else:
        uu = 2.0**-24
        # Per-term FP32 error bound, summed against the oracle's sum of |terms|:
        # the difference z - x carries u (|x| + |z|)/r relative error (doubled
        # in r^2 and again in the kernel), the kernel a few ulps, and the
        # in-tile FP32 accumulation of 256 terms up to 256 u.
        zall = np.concatenate([cy_r, sy_r])
        rmin = np.min(np.linalg.norm(ex_r[:, None, :] - zall[None], axis=2), axis=1)
        zmax = np.linalg.norm(zall, axis=1).max()
        tol = uu * cond * (300 + 4 * (np.linalg.norm(ex_r, axis=1) + zmax) / rmin)
        assert np.all(np.abs(ug - uo) <= tol), np.max(np.abs(ug - uo) / tol)
        # |d2G/dxdn| <= 4/(2 pi r^dim), |dG/dx| <= 1/(2 pi r^(dim-1)) bound the
        # gradient's sum of |terms|
        gsum = (4 * np.abs(a_r).sum() / rmin**dim
                + (np.abs(b_r).sum() + np.abs(sw_r).sum()) / rmin ** (dim - 1)) / (2 * np.pi)
        gtol = uu * gsum * (300 + 6 * (np.linalg.norm(ex_r, axis=1) + zmax) / rmin)
        assert np.all(np.abs(gg - go).max(1) <= gtol + 1e-30)


@pytest.mark.parametrize("dim", [2, 3])
def test_gather_fp32_near_field(B, orc, dim):
    """FP32 gather with the FP64 near field (pairs closer than tau evaluated
    from FP64 copies): matches the FP64 oracle to the FP32 bound of the far
    pairs plus FP64 rounding of the near ones, at evaluation points 1e-6 to
    1e-3 from cache points where the plain FP32 gather is far off."""
    _bvc, pl = B
    say(f"gather fp32 near field dim={dim}")
    ex, cy, cn, a, b, sy, sw = _gather_case(dim, "f32")
    f32 = lambda v: v.astype(np.float32).astype(np.float64)
    cy, cn, a, b, sy, sw = (f32(v) for v in (cy, cn, a, b, sy, sw))  # cache data exact in both precisions
    rng = np.random.default_rng(40 + dim)
    pick = rng.choice(cy.shape[0], 200)
    v = rng.normal(0, 1, (200, dim))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    ex = np.concatenate([ex[:300], cy[pick] + v * (10 ** rng.uniform(-6, -3, 200))[:, None]])
    K = ex.shape[0]
    tau = 1e-2
    dev = lambda x, T: torch.from_numpy(np.ascontiguousarray(x.T if x.ndim == 2 else x)).to("cuda", T)
    F, D = torch.float32, torch.float64
    cache = dict(n=cy.shape[0], dtype=_bvc.F32, x=dev(cy, F), nrm=dev(cn, F), a=dev(a, F), b=dev(b, F))
    src = dict(n=sy.shape[0], dtype=_bvc.F32, y=dev(sy, F), s=dev(sw, F))
    near = dict(tau=tau, x=dev(ex, D), cx=dev(cy, D), cn=dev(cn, D), a=dev(a, D), b=dev(b, D))
    u_n = torch.empty(K, dtype=F, device="cuda")
    g_n = torch.empty(dim, K, dtype=F, device="cuda")
    u_p = torch.empty(K, dtype=F, device="cuda")
    _bvc.bvc_gather_grad(dim, cache, src, K, dev(ex, F), u_n, g_n, near=near)
    _bvc.bvc_gather_u(dim, cache, src, K, dev(ex, F), u_p)
    torch.cuda.synchronize()
    uo, go = orc.gather(dim, ex, cy, cn, a, b, sy, sw, with_grad=True)
    su_far, su_near, sg_far, sg_near, rmin = _abs_terms(dim, ex, cy, cn, a, b, sy, sw, tau)
    x32 = f32(ex)
    uu = 2.0**-24
    zmax = np.linalg.norm(np.concatenate([cy, sy]), axis=1).max()
    # far pairs: the FP32 bound of the plain test, with the FP32 rounding of
    # the evaluation point itself (|x - x32| / r relative per term) added
    shift = np.linalg.norm(ex - x32, axis=1) / rmin
    rel = uu * (300 + 4 * (np.linalg.norm(ex, axis=1) + zmax) / rmin) + 4 * shift
    # plus the FP32 rounding of the result itself (u |value|)
    tol = su_far * rel + 1e-10 * su_near + uu * np.abs(uo)
    err = np.abs(u_n.double().cpu().numpy() - uo)
    assert np.all(err <= tol), np.max(err / tol)
    gtol = sg_far * (rel + 2 * shift) + 1e-10 * sg_near + uu * np.abs(go).max(1)
    gerr = np.abs(to_np_aos(g_n) - go).max(1)
    assert np.all(gerr <= gtol + 1e-30), np.max(gerr / gtol)
    # the points that sit close to a cache point are where the plain FP32
    # gather loses digits and the near field recovers them
    close = np.arange(300, K)[np.linalg.norm(ex[300:] - cy[pick], axis=1) < 1e-4]
    err_p = np.abs(u_p.double().cpu().numpy() - uo)
    assert np.median(err_p[close]) > 10 * np.median(err[close] + 1e-300)


@pytest.mark.parametrize("dim", [2, 3])
def test_gather_backward_fp64(B, orc, dim):
    _bvc, pl = B
    say(f"gather backward dim={dim}")
    ex, cy, cn, a, b, sy, sw = _gather_case(dim, "f64")
    rng = np.random.default_rng(5)
    r = rng.normal(0, 1, ex.shape[0])
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).cuda()
    cache = dict(n=cy.shape[0], dtype=_bvc.F64, x=dev(cy), nrm=dev(cn), a=dev(a), b=dev(b))
    src = dict(n=sy.shape[0], dtype=_bvc.F64, y=dev(sy), s=dev(sw))
    da = torch.empty(cy.shape[0], dtype=torch.float64, device="cuda")
    db = torch.empty_like(da)
    ds = torch.empty(sy.shape[0], dtype=torch.float64, device="cuda")
    dx = torch.empty(dim, ex.shape[0], dtype=torch.float64, device="cuda")
    _bvc.bvc_gather_backward(dim, cache, src, ex.shape[0], dev(ex), dev(r), da, db, ds, dx)
    torch.cuda.synchronize()
    rda, rdb, rds, rdx = orc.gather_backward(dim, ex, r, cy, cn, a, b, sy, sw)
    sc = np.abs(r).sum() * 10
    assert np.allclose(da.cpu().numpy(), rda, rtol=1e-10, atol=1e-12 * sc)
    assert np.allclose(db.cpu().numpy(), rdb, rtol=1e-10, atol=1e-12 * sc)
    assert np.allclose(ds.cpu().numpy(), rds, rtol=1e-10, atol=1e-12 * sc)
    assert np.allclose(to_np_aos(dx), rdx, rtol=1e-9, atol=1e-11 * np.abs(rdx).max())


@pytest.mark.parametrize("case", ["c5", "sphere", "fourier_1", "fourier_5", "sphere_L10"])
def test_basis_means_fp64(B, orc, case):
    _bvc, pl = B
    say(f"basis means {case}")
    if case == "c5":
        p = wl.problem_c5()
        scene, eps, l, sides, n, W = p["scene"], p["eps"], p["offset"], 2, 3000, 8
        basis = wl.fourier_2d(np.zeros(256))
        g = wl.fourier_2d(p["theta_true"])
    elif case.startswith("fourier_"):
        # the smallest bases: the constant alone, and a ragged last chunk
        nb = int(case.split("_")[1])
        p = wl.problem_c5()
        scene, eps, l, sides, n, W = p["scene"], p["eps"], p["offset"], 2, 1500, 8
        basis = wl.fourier_2d(np.zeros(nb))
        g = wl.fourier_2d(np.random.default_rng(9).normal(0, 1, nb))
    elif case == "sphere_L10":
        # beyond the chain kernel's degree: one thread per (cache point, basis)
        scene, eps, l, sides, n, W = wl.displaced_icosphere(2, 3), 4e-3, 2e-2, 1, 200, 4
        basis = wl.solid_harmonics_3d(np.zeros(121), 10)
        g = wl.solid_harmonics_3d(np.random.default_rng(5).normal(0, 1, 121), 10)
    else:
        scene, eps, l, sides, n, W = wl.displaced_icosphere(2, 3), 4e-3, 2e-2, 1, 300, 8
        basis = wl.solid_harmonics_3d(np.zeros(81), 8)
        g = wl.solid_harmonics_3d(np.random.default_rng(4).normal(0, 1, 81), 8)
    sc, gd, _ = _prep(pl, scene, g)
    cache = pl.sample_cache(sc, n, l, sides, 7, 0)
    params = pl.walk_params(eps, W, 17, gd, None, "f64")
    U, D, rec, _ = pl.cache_walks(sc, cache, params, "f64", records=True)
    bd = pl.DeviceField(basis)
    nb = basis.coef.size
    E = torch.empty(cache.n, nb, dtype=torch.float64, device="cuda")
    F = torch.empty_like(E)
    _bvc.bvc_basis_means(bd.c(), scene.dim, cache.n, W, _bvc.F64, rec["exit"], rec["w1"], cache.xbar, 1, E, F)
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    cn = oracle_cache(osc.sample_cache(n, l, sides, 7, 0), cache)
    ref = orc.cache_walks(osc, g, None, orc.walk_params(eps, W, 17), cn, records=True)
    Eo, Fo = orc.basis_means(basis, scene.dim, ref["exit"], ref["w1"], cn["xbar"], W)
    # the device kernel on the oracle's exit records
    E2, F2 = torch.empty_like(E), torch.empty_like(F)
    _bvc.bvc_basis_means(bd.c(), scene.dim, cache.n, W, _bvc.F64, _dev(ref["exit"]), _dev(ref["w1"]),
                         _dev(cn["xbar"]), 1, E2, F2)
    torch.cuda.synchronize()
    assert np.allclose(E2.cpu().numpy(), Eo, rtol=1e-10, atol=1e-11)
    assert np.allclose(F2.cpu().numpy(), Fo, rtol=1e-9, atol=1e-9)
    # the device's own chain: where every walk of a point matches the
    # oracle's, its rows match too
    nW = cache.n * W
    same = (per_walk_match(U.cpu().numpy()[:nW], ref["U"]) & per_walk_match(D.cpu().numpy()[:nW], ref["D"]))
    same = same.reshape(-1, W).all(1)
    assert same.mean() >= 0.99
    assert np.allclose(E.cpu().numpy()[same], Eo[same], rtol=1e-10, atol=1e-11)
    assert np.allclose(F.cpu().numpy()[same], Fo[same], rtol=1e-9, atol=1e-9)
    # linearity: E theta reproduces the walks' own means
    theta = g.coef
    uh = U.cpu().numpy()[:nW].reshape(-1, W).mean(1)
    dh = D.cpu().numpy()[:nW].reshape(-1, W).mean(1)
    assert np.allclose(E.cpu().numpy() @ theta, uh, rtol=1e-9, atol=1e-10)
    assert np.allclose(F.cpu().numpy() @ theta, dh, rtol=1e-8, atol=1e-8)


def test_cache_walks_fp32_statistics(B, orc):
    """FP32 walks follow the FP64 oracle in distribution: per cache point the
    means of independent walk sets (other seeds) agree within 3 standard
    errors, as often as a normal distribution predicts."""
    _bvc, pl = B
    say("cache walks fp32 statistics star_poisson")
    scene, g, f, eps, l, sides, n, W = CASES["star_poisson"]()
    W = 128
    sc, gd, fd = _prep(pl, scene, g, f)
    cache = pl.sample_cache(sc, 1200, l, sides, 3, 0)
    U, D, _, _ = pl.cache_walks(sc, cache, pl.walk_params(eps, W, 11, gd, fd, "f32"), "f32")
    torch.cuda.synchronize()
    osc = orc.Scene(scene)
    ref = orc.cache_walks(osc, g, f, orc.walk_params(eps, W, 12), oracle_cache(osc.sample_cache(1200, l, sides, 3, 0), cache))
    Ug = U.double().cpu().numpy()[: cache.n * W].reshape(-1, W)
    Dg = D.double().cpu().numpy()[: cache.n * W].reshape(-1, W)
    Uo, Do = ref["U"].reshape(-1, W), ref["D"].reshape(-1, W)
    for A, Bo in ((Ug, Uo), (Dg, Do)):
        se = np.sqrt(A.var(1, ddof=1) / W + Bo.var(1, ddof=1) / W) + 1e-12
        z = np.abs(A.mean(1) - Bo.mean(1)) / se
        ok, msg = z_ok(z)
        say(msg)
        assert ok, msg
