"""Pins of the oracle's boundary-data and source fields (not gpu)."""
import numpy as np
import pytest
from scipy.special import exp1

import workloads as wl


def test_ein_against_library(orc):
    """Ein(z) = E1(z) + ln z + gamma, evaluated with 40-digit mpmath (the FP64
    closed form cancels for small z), and against scipy's exp1 for z >= 1."""
    import mpmath

    mpmath.mp.dps = 40
    z = np.concatenate([np.logspace(-8, 3, 200), [0.5, 1.0, 1.999, 2.0, 2.001, 50.0]])
    want = np.array([float(mpmath.e1(v) + mpmath.log(v) + mpmath.euler) for v in z])
    got = np.array([orc.ein(v) for v in z])
    assert np.allclose(got, want, rtol=4e-15, atol=0)
    big = z >= 1
    assert np.allclose(got[big], exp1(z[big]) + np.log(z[big]) + np.euler_gamma, rtol=1e-14)


def test_solid_harmonics_against_scipy(orc):
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, (50, 3))
    r = np.linalg.norm(x, axis=1)
    Y = wl.real_sph_harm(8, x)
    fld = wl.solid_harmonics_3d(np.zeros(81), 8)
    for m in range(81):
        l = int(np.floor(np.sqrt(m)))
        got = orc.basis_eval(fld, 3, m, x)
        assert np.allclose(got, Y[:, m] * r**l, rtol=1e-12, atol=1e-12), m


def _fd_laplacian(orc, fld, x, h=1e-3, with_scale=False):
    dim = x.shape[1]
    f0 = orc.field_eval(fld, x)
    lap = np.zeros(x.shape[0])
    scale = np.zeros(x.shape[0])
    for a in range(dim):
        e = np.zeros(dim)
        e[a] = h
        d2 = orc.field_eval(fld, x + e) + orc.field_eval(fld, x - e) - 2 * f0
        lap += d2
        scale += np.abs(d2)
    return (lap / (h * h), scale / (h * h)) if with_scale else lap / (h * h)


def test_boundary_fields_are_harmonic_or_manufactured(orc):
    rng = np.random.default_rng(2)
    x2 = rng.uniform(-1, 1, (40, 2))
    x3 = rng.uniform(-1, 1, (40, 3))
    assert np.allclose(_fd_laplacian(orc, wl.harmonic_2d(3, 1.0, 1.0), x2), 0, atol=1e-5)
    sh = wl.solid_harmonics_3d(rng.normal(0, 1, 81), 8)
    # the three second differences cancel: Lap is below 1e-5 of their magnitude
    lap, scale = _fd_laplacian(orc, sh, x3, with_scale=True)
    assert np.all(np.abs(lap) <= 1e-5 * scale + 1e-6)
    # a non-harmonic perturbation (one coefficient times |x|^2) would fail it
    assert scale.max() > 1.0
    p = wl.problem_c2(grid=4)
    # Lap of the manufactured g equals the Gaussian source f
    lap = _fd_laplacian(orc, p.g, x2 * 0.8, h=1e-4)
    f = orc.field_eval(p.f, x2 * 0.8)
    assert np.allclose(lap, f, atol=2e-4 * (1 + np.abs(f).max()))


@pytest.mark.parametrize("fld,dim", [
    (wl.harmonic_2d(3, 1.0, 1.0), 2),
    (wl.harmonic_2d(5, -0.5, 2.0), 2),
    (wl.gauss_sum([1.0, -2.0], [[0.1, 0.2], [-0.3, 0.0]], 0.05), 2),
    (wl.gauss_sum([0.7], [[0.1, 0.2, 0.3]], 0.2), 3),
    (wl.fourier_2d(np.random.default_rng(3).normal(0, 1, 256), (0.05, -0.02)), 2),
    (wl.point_source(1.5, [2.0, 0.5]), 2),
    (wl.point_source(-0.5, [2.0, 0.5, 0.1]), 3),
    (wl.solid_harmonics_3d(np.random.default_rng(4).normal(0, 1, 81), 8), 3),
])
def test_fields_match_closed_forms(orc, fld, dim):
    x = np.random.default_rng(5).uniform(-1, 1, (64, dim))
    assert np.allclose(orc.field_eval(fld, x), wl.field_value(fld, x), rtol=1e-12, atol=1e-12)


def test_gauss_potential_closed_form(orc):
    p = wl.problem_c2(grid=4)
    x = np.random.default_rng(6).uniform(-1.2, 1.2, (200, 2))
    assert np.allclose(orc.field_eval(p.g, x), wl.field_value(p.g, x), rtol=1e-12, atol=1e-13)
