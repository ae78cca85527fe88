"""Pins of the oracle's screened Poisson parts (Eq. 1 with sigma > 0,
Appendix A.2), against facts independent of the oracle's arithmetic:

- I0, I1, K0, K1 against scipy.special;
- the free-space Green's function: (Lap - sigma) G = 0 away from the source
  by finite differences, G^sigma - G^0 tends to the constant the delta source
  fixes ((ln(s/2) + gamma)/(2 pi) in 2D, s/(4 pi) in 3D), derivatives against
  central differences, sigma = 0 gives the Poisson kernels;
- the ball weights: for u = exp(a.x) with |a|^2 = sigma (Lap u = sigma u) the
  mean-value factor is u(c) / mean of u over the sphere and the gradient
  factor |grad u(c)| / |mean of nu u over the sphere| (dense quadrature);
- the screened gather (Eqs. 3-6 with G^sigma) reproduces u and grad u at
  interior points from exact boundary data on a circle (trapezoid rule) and a
  sphere (Gauss-Legendre x trapezoid), and a source term on the disk (polar
  quadrature) for u = |x|^2, f = 4 - sigma |x|^2;
- the screened walks' means converge to exp(a.x) and its normal derivative.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle as orc
import workloads as wl


def test_bessel_against_scipy():
    xs = np.concatenate([np.logspace(-8, 0, 40), np.linspace(1.0, 80.0, 120)])
    for name, ref in (("i0", sp.i0), ("i1", sp.i1), ("k0", sp.k0), ("k1", sp.k1)):
        got = np.array([orc.bessel(name, x) for x in xs])
        assert np.allclose(got, ref(xs), rtol=1e-13, atol=0), name


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_greens_function(dim):
    rng = np.random.default_rng(dim)
    sigma = 3.7
    s = np.sqrt(sigma)
    h = 1e-3
    for _ in range(6):
        x = rng.normal(0, 1, dim)
        y = x + rng.normal(0, 1, dim) * 0.6
        ny = rng.normal(0, 1, dim)
        ny /= np.linalg.norm(ny)
        G, dGdx, dGdn, d2 = orc.greens_sigma(dim, sigma, x, y, ny)
        Gx = lambda xx: orc.greens_sigma(dim, sigma, xx, y, ny)[0]
        # (Lap - sigma) G = 0 away from y (fourth-order stencil)
        lap = 0.0
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = h
            lap += (-Gx(x + 2 * e) + 16 * Gx(x + e) - 30 * G + 16 * Gx(x - e) - Gx(x - 2 * e)) / (12 * h * h)
        assert abs(lap - sigma * G) < 1e-6 * (abs(sigma * G) + 1e-3)
        # derivatives against central differences
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = 1e-6
            fd = (Gx(x + e) - Gx(x - e)) / 2e-6
            assert abs(dGdx[a] - fd) < 1e-6 * (1 + abs(fd))
            fdn = (orc.greens_sigma(dim, sigma, x + e, y, ny)[2] - orc.greens_sigma(dim, sigma, x - e, y, ny)[2]) / 2e-6
            assert abs(d2[a] - fdn) < 1e-5 * (1 + abs(fdn))
        Gy = lambda yy: orc.greens_sigma(dim, sigma, x, yy, ny)[0]
        fdy = (Gy(y + 1e-6 * ny) - Gy(y - 1e-6 * ny)) / 2e-6
        assert abs(dGdn - fdy) < 1e-6 * (1 + abs(fdy))
        # sigma = 0 is the Poisson kernel
        p0 = orc.greens(dim, x, y, ny)
        z0 = orc.greens_sigma(dim, 0.0, x, y, ny)
        assert z0[0] == p0[0] and z0[2] == p0[2] and np.array_equal(z0[1], p0[1]) and np.array_equal(z0[3], p0[3])
    # the delta normalisation: G^sigma - G^0 -> constant as r -> 0
    x = np.zeros(dim)
    y = np.zeros(dim)
    y[0] = 1e-7
    diff = orc.greens_sigma(dim, sigma, x, y)[0] - orc.greens(dim, x, y)[0]
    want = (np.log(s / 2) + np.euler_gamma) / (2 * np.pi) if dim == 2 else s / (4 * np.pi)
    assert abs(diff - want) < 1e-6


def _sphere_quadrature(dim, n):
    """Nodes, weights of the unit circle / sphere (trapezoid; Gauss-Legendre in
    cos(theta) x trapezoid in phi)."""
    if dim == 2:
        t = 2 * np.pi * (np.arange(n) + 0.5) / n
        return np.stack([np.cos(t), np.sin(t)], 1), np.full(n, 2 * np.pi / n)
    zq, wq = np.polynomial.legendre.leggauss(n)
    ph = 2 * np.pi * (np.arange(2 * n) + 0.5) / (2 * n)
    Z, P = np.meshgrid(zq, ph, indexing="ij")
    rho = np.sqrt(1 - Z**2)
    pts = np.stack([rho * np.cos(P), rho * np.sin(P), Z], -1).reshape(-1, 3)
    w = (wq[:, None] * np.full(2 * n, 2 * np.pi / (2 * n))[None]).ravel()
    return pts, w


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_ball_weights(dim):
    sigma = 2.3
    a = np.ones(dim) / np.sqrt(dim) * np.sqrt(sigma)
    c = np.array([0.2, -0.1, 0.05][:dim])
    nu, w = _sphere_quadrature(dim, 200 if dim == 2 else 40)
    area = w.sum()
    for R in (0.05, 0.4, 1.7):
        z = c + R * nu
        uz = np.exp(z @ a)
        uc = np.exp(c @ a)
        P = uc / (np.sum(w * uz) / area)
        assert orc.screen_ball_weight(dim, sigma, R) == pytest.approx(P, rel=1e-11)
        m = np.sum(w[:, None] * nu * uz[:, None], 0) / area
        grad = a * uc
        assert orc.screen_grad_weight(dim, sigma, R) == pytest.approx(np.linalg.norm(grad) / np.linalg.norm(m),
                                                                     rel=1e-10)
        assert orc.screen_ball_weight(dim, 0.0, R) == 1.0
        assert orc.screen_grad_weight(dim, 0.0, R) == pytest.approx(dim / R)


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_gather_reproduces_solution(dim):
    sigma = 1.9
    a = np.array([0.8, -0.5, 0.3][:dim])
    a = a / np.linalg.norm(a) * np.sqrt(sigma)
    z, w = _sphere_quadrature(dim, 400 if dim == 2 else 60)
    u = np.exp(z @ a)
    dudn = u * (z @ a)  # outward normal of the unit ball is z
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (20, dim))
    x *= (0.6 * rng.random(20) ** (1 / dim) / np.linalg.norm(x, axis=1))[:, None]
    got_u, got_g = orc.gather_sigma(dim, sigma, x, z, z, u * w, dudn * w)
    ux = np.exp(x @ a)
    assert np.allclose(got_u, ux, rtol=1e-9, atol=1e-10)
    assert np.allclose(got_g, a[None] * ux[:, None], rtol=1e-8, atol=1e-9)
    # sigma = 0 gives the plain gather
    p0 = orc.gather(dim, x, z, z, u * w, dudn * w)
    q0 = orc.gather_sigma(dim, 0.0, x, z, z, u * w, dudn * w)
    assert np.array_equal(p0[0], q0[0]) and np.array_equal(p0[1], q0[1])


def test_screened_gather_source_term_on_the_disk():
    """(Lap - sigma) u = f with u = |x|^2, f = 4 - sigma |x|^2 on the unit disk:
    boundary terms (u = 1, du/dn = 2) plus the source term by polar
    Gauss-Legendre x trapezoid quadrature reproduce u(x)."""
    sigma = 2.6
    z, w = _sphere_quadrature(2, 600)
    rq, wr = np.polynomial.legendre.leggauss(120)
    r = 0.5 * (rq + 1)
    wr = 0.5 * wr
    t = 2 * np.pi * (np.arange(240) + 0.5) / 240
    R, T = np.meshgrid(r, t, indexing="ij")
    y = np.stack([R * np.cos(T), R * np.sin(T)], -1).reshape(-1, 2)
    wy = (wr[:, None] * R * (2 * np.pi / 240)).ravel()
    f = 4 - sigma * np.sum(y * y, 1)
    x = np.array([[0.1, 0.2], [-0.35, 0.0], [0.0, -0.5]])
    got = orc.gather_sigma(2, sigma, x, z, z, np.ones(z.shape[0]) * w, 2 * w, y, f * wy, with_grad=False)
    # the polar grid is centred at 0, not at x, so the log singularity of G
    # limits the volume quadrature to about 1e-4
    assert np.allclose(got, np.sum(x * x, 1), atol=2e-4)
    # the source term carries the screening: with sigma = 0 the same data miss
    bad = orc.gather_sigma(2, 0.0, x, z, z, np.ones(z.shape[0]) * w, 2 * w, y, f * wy, with_grad=False)
    assert np.all(np.abs(bad - np.sum(x * x, 1)) > 1e-2)


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_walks_converge(dim):
    """Pointwise walks (u and grad u) and cache-mode walks (n . grad u) of
    Lap u = sigma u with g = exp(a.x), which solves the PDE everywhere, so the
    polygonal or triangulated domain changes nothing: walk means must match
    exp(a.x) and a exp(a.x) within their standard errors (eps = 1e-4)."""
    sigma = 4.0
    a = np.array([1.0, 0.6, -0.4][:dim])
    a = a / np.linalg.norm(a) * np.sqrt(sigma)
    g = wl.exp_plane(1.0, a)
    scene = wl.circle_polygon(256) if dim == 2 else wl.icosphere(3)
    osc = orc.Scene(scene)
    P = orc.walk_params(1e-4, 1, 2024, sigma=sigma)
    rng = np.random.default_rng(dim)
    W = 1500
    for i in range(4):
        v = rng.normal(0, 1, dim)
        v /= np.linalg.norm(v)
        x = v * (0.3 + 0.15 * i)
        n = v  # a unit direction for the normal-derivative weight
        d, xb, _ = osc.closest(x)
        us, gs, ds = [], [], []
        for j in range(W):
            w1 = orc.walk(osc, g, None, P, 1, x, None, d[0], xb[0], i * W + j)
            us.append(w1["U"])
            gs.append(w1["grad"])
            w0 = orc.walk(osc, g, None, P, 0, x, n, d[0], xb[0], i * W + j)
            ds.append(float(np.dot(n, w0["grad"])))
        us, gs, ds = np.array(us), np.array(gs), np.array(ds)
        ux = np.exp(x @ a)
        se = lambda v: v.std(ddof=1) / np.sqrt(v.size)
        assert abs(us.mean() - ux) < 5 * se(us) + 1e-3 * ux
        for q in range(dim):
            assert abs(gs[:, q].mean() - a[q] * ux) < 5 * se(gs[:, q]) + 2e-3 * ux
        assert abs(ds.mean() - n @ a * ux) < 5 * se(ds) + 2e-3 * ux
        assert us.std() > 0  # the weights vary walk to walk

