"""Pins of the oracle's Green's functions and gather (not gpu).

The kernels of Appendix A.1 are pinned by finite differences, harmonicity and
the Gauss identity; the gather (Eqs. 3-6) by exact boundary data on a circle,
where the periodic trapezoid rule makes the boundary-integral sum converge to
machine precision; the 3D sign of G by the sphere with u = x_1.
"""
import numpy as np
import pytest

import workloads as wl


def _rand_pairs(rng, dim, n):
    x = rng.normal(0, 1, (n, dim))
    y = rng.normal(0, 1, (n, dim))
    nn = rng.normal(0, 1, (n, dim))
    nn /= np.linalg.norm(nn, axis=1, keepdims=True)
    return x, y, nn


@pytest.mark.parametrize("dim", [2, 3])
def test_greens_derivatives_finite_differences(orc, dim):
    rng = np.random.default_rng(dim)
    h = 1e-6
    for x, y, nn in zip(*_rand_pairs(rng, dim, 20)):
        G, dGdx, dGdn, d2 = orc.greens(dim, x, y, nn)
        fd_dx = np.zeros(dim)
        fd_d2 = np.zeros(dim)
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = h
            fd_dx[a] = (orc.greens(dim, x + e, y, nn)[0] - orc.greens(dim, x - e, y, nn)[0]) / (2 * h)
            fd_d2[a] = (orc.greens(dim, x + e, y, nn)[2] - orc.greens(dim, x - e, y, nn)[2]) / (2 * h)
        fd_dn = (orc.greens(dim, x, y + h * nn, nn)[0] - orc.greens(dim, x, y - h * nn, nn)[0]) / (2 * h)
        sc = 1 + np.abs(dGdx).max()
        assert np.allclose(dGdx, fd_dx, atol=1e-7 * sc)
        assert abs(dGdn - fd_dn) < 1e-7 * (1 + abs(dGdn))
        assert np.allclose(d2, fd_d2, atol=1e-6 * (1 + np.abs(d2).max()))


@pytest.mark.parametrize("dim", [2, 3])
def test_greens_is_harmonic_with_unit_flux(orc, dim):
    """Lap G = 0 away from the pole, and the flux of grad_x G through a sphere
    around y is 1 (Lap G = delta, the sign convention of Eq. 2)."""
    rng = np.random.default_rng(10 + dim)
    h = 1e-4
    for _ in range(10):
        x = rng.normal(0, 1, dim)
        y = rng.normal(0, 1, dim)
        lap = 0.0
        g0 = orc.greens(dim, x, y)[0]
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = h
            lap += orc.greens(dim, x + e, y)[0] + orc.greens(dim, x - e, y)[0] - 2 * g0
        lap /= h * h
        assert abs(lap) < 1e-4 * (1 + abs(g0))
    # flux of grad_x G over a small sphere around y
    y = np.zeros(dim)
    if dim == 2:
        m = 2000
        th = 2 * np.pi * (np.arange(m) + 0.5) / m
        pts = 0.3 * np.stack([np.cos(th), np.sin(th)], 1)
        wts = np.full(m, 2 * np.pi * 0.3 / m)
    else:
        m = 20000
        k = np.arange(m) + 0.5
        z = 1 - 2 * k / m
        ph = np.pi * (1 + 5**0.5) * k
        pts = 0.3 * np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z], 1)
        wts = np.full(m, 4 * np.pi * 0.09 / m)
    flux = sum(w * np.dot(orc.greens(dim, p, y)[1], p / 0.3) for p, w in zip(pts, wts))
    assert abs(flux - 1.0) < 1e-3


def _circle_cache(N):
    th = 2 * np.pi * (np.arange(N) + 0.5) / N
    y = np.stack([np.cos(th), np.sin(th)], 1)
    return y, y.copy(), np.full(N, 2 * np.pi / N)


def test_gauss_identity_2d(orc):
    y, n, w = _circle_cache(4096)
    ex = np.array([[0.1, 0.2], [-0.5, 0.3], [0.0, 0.0], [1.5, 0.2]])
    # u = 1: dG/dn summed over the boundary is 1 inside, 0 outside
    u = orc.gather(2, ex, y, n, w, np.zeros_like(w), with_grad=False)
    assert np.allclose(u, [1, 1, 1, 0], atol=1e-12)


def test_exact_cache_gather_2d(orc):
    """Eq. 3 and Eq. 5 with exact u and du/dn on the unit circle reproduce the
    harmonic solution u = Re z^3 + e^x cos y and its gradient."""
    g = wl.harmonic_2d(3, 1.0, 1.0)
    y, n, w = _circle_cache(1024)
    u = wl.field_value(g, y)
    grad = wl.field_grad_fd(g, y, 1e-6)
    # exact normal derivative from the analytic gradient
    z = y[:, 0] + 1j * y[:, 1]
    dz = 3 * z**2  # d/dz of z^3; grad Re f = (Re f', -Im f')
    gx = dz.real + np.exp(y[:, 0]) * np.cos(y[:, 1])
    gy = -dz.imag - np.exp(y[:, 0]) * np.sin(y[:, 1])
    assert np.allclose(np.stack([gx, gy], 1), grad, atol=1e-8)
    dudn = gx * n[:, 0] + gy * n[:, 1]
    ex = np.array([[0.1, 0.2], [-0.5, 0.3], [0.0, 0.0], [0.6, -0.6]])
    uk, gk = orc.gather(2, ex, y, n, u * w, dudn * w)
    assert np.allclose(uk, wl.field_value(g, ex), atol=1e-12)
    z = ex[:, 0] + 1j * ex[:, 1]
    want = np.stack([(3 * z**2).real + np.exp(ex[:, 0]) * np.cos(ex[:, 1]),
                     -(3 * z**2).imag - np.exp(ex[:, 0]) * np.sin(ex[:, 1])], 1)
    assert np.allclose(gk, want, atol=1e-11)


def _fibonacci_sphere(N):
    k = np.arange(N) + 0.5
    z = 1 - 2 * k / N
    ph = np.pi * (1 + 5**0.5) * k
    p = np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z], 1)
    return p, p.copy(), np.full(N, 4 * np.pi / N)


def test_exact_cache_gather_3d_fixes_sign_of_g(orc):
    """u = x_1 on the unit sphere: with G = -1/(4 pi r) the boundary integral
    returns 0.2 at x = (0.2, -0.1, 0.3); the printed +1/(4 pi r) would give 0.0667."""
    y, n, w = _fibonacci_sphere(200000)
    ex = np.array([[0.2, -0.1, 0.3], [0.0, 0.0, 0.0], [-0.3, 0.4, 0.1]])
    u = y[:, 0]
    dudn = n[:, 0]
    uk, gk = orc.gather(3, ex, y, n, u * w, dudn * w)
    assert np.allclose(uk, ex[:, 0], atol=2e-4)
    assert np.allclose(gk, [[1, 0, 0]] * 3, atol=2e-3)
    # Gauss identity in 3D
    one = orc.gather(3, ex, y, n, w, np.zeros_like(w), with_grad=False)
    assert np.allclose(one, 1.0, atol=2e-4)


def test_source_term_disk_closed_form(orc):
    """Eq. 4: int_D G(x, y) dy = (|x|^2 - 1)/4 on the unit disk (Lap = 1, zero on
    the circle); estimated with uniform source samples."""
    rng = np.random.default_rng(4)
    M = 400000
    r = np.sqrt(rng.random(M))
    t = 2 * np.pi * rng.random(M)
    sy = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    sw = np.full(M, np.pi / M)
    ex = np.array([[0.1, 0.2], [-0.5, 0.3], [0.7, 0.0]])
    u, gr = orc.gather(2, ex, np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(0), np.zeros(0), sy, sw)
    want = ((ex**2).sum(1) - 1) / 4
    assert np.allclose(u, want, atol=3e-3)
    assert np.allclose(gr, ex / 2, atol=3e-2)  # Eq. 6: gradient of (|x|^2-1)/4
