"""Statistical pins of the oracle's walks and cache sampler (not gpu).

Walk on spheres (Section 3.1) and the ball gradient estimator (Eq. 7) are
checked in expectation against closed forms: the harmonic measure of the disk
(Poisson kernel), harmonic and manufactured Poisson solutions, and the ball
gradient identity.  Tolerances: 4 standard errors plus the epsilon-shell bias
bound eps * max|grad u| (the walk stops within eps of the boundary and reads g
at the closest point).
"""
import numpy as np
import pytest
from scipy import stats

import workloads as wl


def _disk(n=2048):
    return wl.circle_polygon(n)


def test_exit_distribution_is_poisson_kernel(orc):
    sc = orc.Scene(_disk(4096))
    x0 = np.array([0.3, 0.2])
    d, xb, _ = sc.closest(x0)
    P = orc.walk_params(1e-5, 1, seed=77)
    th = []
    for i in range(12000):
        r = orc.walk(sc, wl.Field(), None, P, 1, x0, None, d[0], xb[0], i)
        th.append(np.arctan2(r["exit"][1], r["exit"][0]))
    th = np.mod(np.array(th), 2 * np.pi)
    # harmonic measure of the unit disk seen from x0
    z0 = complex(*x0)

    def cdf(t):
        t = np.atleast_1d(t)
        grid = np.linspace(0, 2 * np.pi, 20001)
        pk = (1 - abs(z0) ** 2) / (2 * np.pi * np.abs(np.exp(1j * grid) - z0) ** 2)
        c = np.concatenate([[0], np.cumsum((pk[1:] + pk[:-1]) / 2 * np.diff(grid))])
        return np.interp(t, grid, c / c[-1])

    assert stats.kstest(th, cdf).pvalue > 1e-3


def test_pointwise_harmonic_mean_value(orc):
    p = wl.problem_c1()
    sc = orc.Scene(p.scene)
    rng = np.random.default_rng(3)
    r = 0.9 * np.sqrt(rng.random(24))
    t = 2 * np.pi * rng.random(24)
    x = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    W = 2000
    P = orc.walk_params(p.eps, W, seed=5)
    u, gr, steps = orc.pointwise(sc, p.g, None, P, x)
    # per-walk spread, measured from an independent batch
    u_b, _, _ = orc.pointwise(sc, p.g, None, orc.walk_params(p.eps, W, seed=6), x)
    sem = np.std(u - u_b) / np.sqrt(2)
    truth = wl.field_value(p.g, x)
    bias = p.eps * 6.0  # |grad g| <= ~6 on the unit disk
    assert np.all(np.abs(u - truth) <= 4.5 * sem + bias)
    assert steps > 0


def test_ball_gradient_identity_harmonic(orc):
    """E[(dim/R) nu u(x + R nu)] = grad u(x) for harmonic u (cache walk mode)."""
    sc = orc.Scene(_disk(2048))
    g = wl.harmonic_2d(3, 1.0, 1.0)
    x = np.array([0.2, -0.1])
    d, xb, _ = sc.closest(x)
    P = orc.walk_params(1e-4, 1, seed=9, control_variate=True)
    n = np.array([1.0, 0.0])
    G = np.array([orc.walk(sc, g, None, P, 0, x, n, d[0], xb[0], i)["grad"] for i in range(20000)])
    want = wl.field_grad_fd(g, x[None, :])[0]
    sem = G.std(0) / np.sqrt(G.shape[0])
    assert np.all(np.abs(G.mean(0) - want) < 4.5 * sem + 1e-3)


def test_poisson_walk_and_gradient_manufactured(orc):
    """Poisson (Lap u = f) with the manufactured Gaussian-potential solution:
    the in-walk source terms (density |G^B|) and the 2D gradient source term
    (radius density (3/2)(1 - s^2)) give unbiased u and grad u."""
    amps, centers, sigma = np.array([3.0, -2.0]), np.array([[0.1, 0.1], [-0.2, 0.15]]), 0.15
    f = wl.gauss_sum(amps, centers, sigma)
    g = wl.gauss_potential_2d(amps, centers, sigma, 3, 1.0, 1.0)
    sc = orc.Scene(_disk(2048))
    x = np.array([0.05, 0.12])
    d, xb, _ = sc.closest(x)
    P = orc.walk_params(1e-4, 1, seed=21)
    res = [orc.walk(sc, g, f, P, 0, x, np.array([0.0, 1.0]), d[0], xb[0], i) for i in range(20000)]
    U = np.array([r["U"] for r in res])
    G = np.array([r["grad"] for r in res])
    u_true = wl.field_value(g, x[None, :])[0]
    g_true = wl.field_grad_fd(g, x[None, :], 1e-6)[0]
    assert abs(U.mean() - u_true) < 4.5 * U.std() / np.sqrt(U.size) + 1e-3
    semg = G.std(0) / np.sqrt(G.shape[0])
    assert np.all(np.abs(G.mean(0) - g_true) < 4.5 * semg + 1e-3)
    # dropping the in-ball source term biases u by far more than the noise
    no_src = np.array([orc.walk(sc, g, None, P, 0, x, None, d[0], xb[0], i)["U"] for i in range(4000)])
    assert abs(no_src.mean() - u_true) > 5 * U.std() / np.sqrt(U.size)


def test_capped_walks_are_flagged(orc):
    sc = orc.Scene(_disk(256))
    x = np.array([0.0, 0.0])
    d, xb, _ = sc.closest(x)
    # the first ball lands within 7.5e-5 of the 256-gon, so use a thinner shell
    P = orc.walk_params(1e-8, 1, seed=1, max_steps=1)
    r = orc.walk(sc, wl.harmonic_2d(), None, P, 0, x, None, d[0], xb[0], 0)
    assert r["capped"] and r["steps"] == 1


def test_control_variate_keeps_mean_and_cuts_variance(orc):
    p = wl.problem_c1()
    sc = orc.Scene(p.scene)
    cache = sc.sample_cache(64, 5e-3, 1, seed=31)
    keep = cache["accept"]
    cache = {k: v[keep] for k, v in cache.items() if isinstance(v, np.ndarray)}
    W = 400
    on = orc.cache_walks(sc, p.g, None, orc.walk_params(p.eps, W, 3, control_variate=True), cache)
    off = orc.cache_walks(sc, p.g, None, orc.walk_params(p.eps, W, 3, control_variate=False), cache)
    Don = on["D"].reshape(-1, W)
    Doff = off["D"].reshape(-1, W)
    # same walks, so the difference of the means is (dim/R0) mean(nu.n) c: zero-mean
    diff = Don.mean(1) - Doff.mean(1)
    sem = np.sqrt(Doff.var(1) / W)
    assert np.mean(np.abs(diff) < 4.5 * sem) > 0.95
    assert Don.var(1).mean() < 0.2 * Doff.var(1).mean()
    # U does not depend on the control variate
    assert np.array_equal(on["U"], off["U"])


def test_cache_estimates_match_closed_form(orc):
    """u-hat and du/dn-hat at cache points on the offset boundary l = 5 eps."""
    p = wl.problem_c1()
    sc = orc.Scene(p.scene)
    l = 5 * p.eps
    cache = sc.sample_cache(48, l, 1, seed=41)
    keep = cache["accept"]
    cache = {k: v[keep] for k, v in cache.items() if isinstance(v, np.ndarray)}
    W = 1500
    out = orc.cache_walks(sc, p.g, None, orc.walk_params(p.eps, W, 8), cache)
    U = out["U"].reshape(-1, W)
    D = out["D"].reshape(-1, W)
    uh, dh = orc.reduce(out["U"], out["D"], W)
    assert np.allclose(uh, U.mean(1)) and np.allclose(dh, D.mean(1))
    u_true = wl.field_value(p.g, cache["x"])
    grad = wl.field_grad_fd(p.g, cache["x"])
    dn_true = (grad * cache["n"]).sum(1)
    assert np.all(np.abs(uh - u_true) < 4.5 * U.std(1) / np.sqrt(W) + p.eps * 6)
    # the normal derivative carries the epsilon-shell bias of a ball of radius
    # l = 5 eps: first order it inflates |du/dn| by a few percent
    err = dh - dn_true
    assert np.mean(np.abs(err) < 4.5 * D.std(1) / np.sqrt(W) + 0.1 * np.abs(dn_true) + 0.05) > 0.95


def test_offset_cache_sampler_circle(orc):
    p = wl.problem_c1()
    sc = orc.Scene(p.scene)
    l = 5e-3
    n = 4096
    c = sc.sample_cache(n, l, 1, seed=51)
    acc = c["accept"]
    assert np.allclose(c["R0"][acc], l, rtol=1e-9)
    assert np.allclose(np.linalg.norm(c["n"], axis=1), 1, atol=1e-12)
    assert np.all(sc.inside(c["x"][acc]) != 0)
    # total accepted weight estimates the length of the inner offset polygon
    m = 128
    apothem = np.cos(np.pi / m)
    want = 2 * m * (apothem - l) * np.tan(np.pi / m)
    got = c["w"][acc].sum()
    assert abs(got - want) < 2e-3 * want
    # uniform by arclength: angles of accepted points are uniform
    th = np.mod(np.arctan2(c["x"][acc, 1], c["x"][acc, 0]), 2 * np.pi)
    assert stats.kstest(th, lambda t: t / (2 * np.pi)).pvalue > 1e-3
    # the measure is the sum of segment lengths and vertex circles
    seg = np.linalg.norm(np.diff(np.vstack([p.scene.verts, p.scene.verts[:1]]), axis=0), axis=1).sum()
    assert abs(sc.candidate_measure(l, 1) - (seg + m * 2 * np.pi * l)) < 1e-12


def test_offset_cache_sampler_sphere(orc):
    sph = wl.icosphere(3)
    sc = orc.Scene(sph)
    l = 0.01
    c = sc.sample_cache(8192, l, 1, seed=61)
    acc = c["accept"]
    assert np.allclose(c["R0"][acc], l, rtol=1e-9)
    assert np.all(sc.inside(c["x"][acc]) == 1)
    # the offset surface of a convex polyhedron moved inward has the area of the
    # faces' inner parallel surface, slightly below the mesh area
    a, b, cc = (sph.verts[sph.prims[:, k]] for k in range(3))
    area = 0.5 * np.linalg.norm(np.cross(b - a, cc - a), axis=1).sum()
    got = c["w"][acc].sum()
    assert area * (1 - 3 * l) < got < area * (1 + 1e-3)


def test_offset_sampler_star_both_sides(orc):
    p = wl.problem_c2(grid=4)
    sc = orc.Scene(p.scene)
    c = sc.sample_cache(16384, p.offset, 2, seed=71)
    acc = c["accept"]
    # the self-intersecting band is denser than 2 l, so most of the candidate
    # measure is closer than l to another segment and is rejected
    assert 0.005 < acc.mean() < 0.2
    d, _, _ = sc.closest(c["x"][~acc][:500])
    assert np.all((d < p.offset * (1 - 1e-9)) | (sc.inside(c["x"][~acc][:500]) == 0))
    assert np.allclose(c["R0"][acc], p.offset, rtol=1e-9)
    assert np.all(sc.inside(c["x"][acc]) != 0)


def test_source_sampler_measures_region(orc):
    sc = orc.Scene(wl.circle_polygon(512))
    l = 0.01
    y, sw = sc.sample_sources(wl.Field(1, [], [1.0]), 128, [-1, -1], [1, 1], l, seed=81)
    # with f = 1 the weights add up to the area of {d > l} inside the polygon
    want = np.pi * (np.cos(np.pi / 512) - l) ** 2 * (512 * np.sin(2 * np.pi / 512) / 2) / np.pi
    assert abs(sw.sum() - want) < 5e-3 * want
