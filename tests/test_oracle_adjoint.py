"""Pins of the oracle's adjoints and basis expansions (not gpu).

Every estimator of Eqs. 3-6 is linear in the cache values (a, b) and source
weights (s); the transposed gather must equal J^T r for the Jacobian assembled
column by column from forward gathers, and dL/dx must equal r * grad u (the
gradient of Eq. 5, checked by finite differences).  The basis means of the walk
exit records must reproduce, by linearity, the walks run with the full field.
"""
import numpy as np

import workloads as wl


def _small_problem(rng, dim):
    K, N, M = 7, 11, 5
    ex = rng.normal(0, 0.3, (K, dim))
    th = rng.normal(0, 1, (N, dim))
    cy = th / np.linalg.norm(th, axis=1, keepdims=True)
    cn = cy.copy()
    a = rng.normal(0, 1, N)
    b = rng.normal(0, 1, N)
    sy = rng.normal(0, 0.5, (M, dim))
    sw = rng.normal(0, 1, M)
    return ex, cy, cn, a, b, sy, sw


def test_gather_backward_is_transposed_jacobian(orc):
    for dim in (2, 3):
        rng = np.random.default_rng(dim)
        ex, cy, cn, a, b, sy, sw = _small_problem(rng, dim)
        r = rng.normal(0, 1, ex.shape[0])
        da, db, ds, dx = orc.gather_backward(dim, ex, r, cy, cn, a, b, sy, sw)
        N, M = a.size, sw.size
        Ja = np.stack([orc.gather(dim, ex, cy, cn, np.eye(N)[i], 0 * b, sy, 0 * sw, with_grad=False)
                       for i in range(N)], 1)
        Jb = np.stack([orc.gather(dim, ex, cy, cn, 0 * a, np.eye(N)[i], sy, 0 * sw, with_grad=False)
                       for i in range(N)], 1)
        Js = np.stack([orc.gather(dim, ex, cy, cn, 0 * a, 0 * b, sy, np.eye(M)[j], with_grad=False)
                       for j in range(M)], 1)
        assert np.allclose(da, Ja.T @ r, rtol=1e-12, atol=1e-12)
        assert np.allclose(db, Jb.T @ r, rtol=1e-12, atol=1e-12)
        assert np.allclose(ds, Js.T @ r, rtol=1e-12, atol=1e-12)
        # position adjoint against central differences of the forward gather
        h = 1e-6
        fd = np.zeros_like(ex)
        for k in range(ex.shape[0]):
            for q in range(dim):
                e = np.zeros_like(ex)
                e[k, q] = h
                up = orc.gather(dim, ex + e, cy, cn, a, b, sy, sw, with_grad=False)
                dn = orc.gather(dim, ex - e, cy, cn, a, b, sy, sw, with_grad=False)
                fd[k, q] = r[k] * (up[k] - dn[k]) / (2 * h)
        assert np.allclose(dx, fd, rtol=1e-6, atol=1e-7)


def test_basis_means_reproduce_walks_2d_fourier(orc):
    p = wl.problem_c5()
    sc = orc.Scene(p["scene"])
    cache = sc.sample_cache(3000, p["offset"], 2, seed=5)
    keep = cache["accept"]
    cache = {k: v[keep] for k, v in cache.items() if isinstance(v, np.ndarray)}
    W = 16
    theta = p["theta_true"]
    g = wl.fourier_2d(theta, (0.0, 0.0))
    P = orc.walk_params(p["eps"], W, seed=p["seed_walks"])
    out = orc.cache_walks(sc, g, None, P, cache, records=True)
    uh, dh = orc.reduce(out["U"], out["D"], W)
    E, F = orc.basis_means(wl.fourier_2d(np.zeros(256)), 2, out["exit"], out["w1"], cache["xbar"], W)
    assert np.allclose(E @ theta, uh, rtol=1e-10, atol=1e-12)
    assert np.allclose(F @ theta, dh, rtol=1e-9, atol=1e-10)


def test_basis_means_reproduce_walks_3d_harmonics(orc):
    sph = wl.displaced_icosphere(2, 11)
    sc = orc.Scene(sph)
    cache = sc.sample_cache(200, 0.02, 1, seed=6)
    keep = cache["accept"]
    cache = {k: v[keep] for k, v in cache.items() if isinstance(v, np.ndarray)}
    W = 8
    coef = np.random.default_rng(2).normal(0, 1, 81)
    g = wl.solid_harmonics_3d(coef, 8)
    out = orc.cache_walks(sc, g, None, orc.walk_params(0.004, W, seed=3), cache, records=True)
    uh, dh = orc.reduce(out["U"], out["D"], W)
    E, F = orc.basis_means(wl.solid_harmonics_3d(np.zeros(81), 8), 3, out["exit"], out["w1"],
                           cache["xbar"], W)
    assert np.allclose(E @ coef, uh, rtol=1e-10, atol=1e-11)
    assert np.allclose(F @ coef, dh, rtol=1e-9, atol=1e-9)
