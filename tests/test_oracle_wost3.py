"""Pins of the oracle's walk on stars in 3D and of its Neumann term (h != 0,
2D and 3D), against facts independent of the oracle's arithmetic:

- silhouettes of a box tube seen from inside: with Dirichlet faces x = +-1
  and Neumann faces y = +-1, z = +-1 (each face a grid of triangles), no
  edge inside a face (flat) and no edge of the convex tube hides anything,
  so the silhouette distance is the distance to the two square frames where
  the Neumann part ends, sqrt((1 -+ x)^2 + (1 - max(|y|, |z|))^2); a point on
  the face y = -1 sees that face edge-on, so the tube edges of that face
  count too (distance 1 - |z|);
- u = x on that box (zero flux through the Neumann faces): walk means from
  interior points and from points on a Neumann face equal x within their
  standard errors;
- u = x^2 - y^2 with Neumann faces y = +-1 (h = du/dn = -2 on both) and
  Dirichlet data elsewhere, in 2D (the square) and 3D (the box): the walks'
  Neumann terms are what makes the means right; without them the means miss
  by more than 20 standard errors at the interior points used here;
- the first-ball gradient (mode 0) at offset Dirichlet points of the box:
  n . grad u = 1 for u = x.
"""
import numpy as np

import oracle as orc
import workloads as wl


def _se(v):
    return v.std(ddof=1) / np.sqrt(v.size)


def _box(neumann, m=4):
    full, dir_, neu = wl.mixed_box((-1, -1, -1), (1, 1, 1), neumann, m)
    return full, orc.Scene(dir_), orc.Scene(neu)


def _sh(fn, lmax=2):
    """Solid-harmonic coefficients reproducing the harmonic polynomial fn."""
    rng = np.random.default_rng(0)
    x = rng.normal(0, 1, (200, 3))
    Y = wl.real_sph_harm(lmax, x)
    ls = np.array([l for l in range(lmax + 1) for _ in range(2 * l + 1)])
    A = Y * np.linalg.norm(x, axis=1)[:, None] ** ls[None, :]
    c, *_ = np.linalg.lstsq(A, fn(x), rcond=None)
    c[np.abs(c) < 1e-12] = 0
    f = wl.solid_harmonics_3d(c, lmax)
    assert np.allclose(wl.field_value(f, x), fn(x), atol=1e-12)
    return f


TUBE = [False, False, True, True, True, True]  # Neumann on y and z faces


def test_box_tube_silhouettes():
    _, _, on = _box(TUBE)
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.95, 0.95, (200, 3))
    d = orc.silhouette_distances(on, x)
    m = 1 - np.maximum(np.abs(x[:, 1]), np.abs(x[:, 2]))
    ref = np.minimum(np.hypot(1 - x[:, 0], m), np.hypot(1 + x[:, 0], m))
    assert np.allclose(d, ref, rtol=0, atol=1e-12)
    # on the face y = -1
    f = np.stack([rng.uniform(-0.9, 0.9, 50), -np.ones(50), rng.uniform(-0.9, 0.9, 50)], 1)
    d = orc.silhouette_distances(on, f)
    ref = np.minimum(np.minimum(1 - f[:, 0], 1 + f[:, 0]), 1 - np.abs(f[:, 2]))
    assert np.allclose(d, ref, rtol=0, atol=1e-12)


def test_box_tube_u_equals_x():
    _, od, on = _box(TUBE)
    g = _sh(lambda x: x[:, 0], 1)
    W = 1500
    P = orc.walk_params(1e-3, W, 21)
    pts = np.array([[0.3, 0.1, -0.2], [-0.7, 0.6, 0.5], [0.85, -0.3, 0.7]])
    U, _, _ = orc.wost_walks(od, on, g, P, 1, pts)
    U = U.reshape(len(pts), W)
    for i in range(len(pts)):
        assert abs(U[i].mean() - pts[i, 0]) <= 4 * _se(U[i]) + 2e-3
    # from points on the Neumann face z = 1 (outward normal +z)
    f = np.array([[0.2, -0.4, 1.0], [-0.5, 0.3, 1.0]])
    U, _, _ = orc.wost_walks(od, on, g, P, 3, f, nrm=np.array([[0, 0, 1.0]] * 2))
    U = U.reshape(len(f), W)
    for i in range(len(f)):
        assert abs(U[i].mean() - f[i, 0]) <= 4 * _se(U[i]) + 2e-3


def _check_neumann_data(od, on, g, h, P, pts, nrm, mode, truth):
    W = P.n_walks
    U, _, _ = orc.wost_walks(od, on, g, P, mode, pts, nrm=nrm, h=h)
    U0, _, _ = orc.wost_walks(od, on, g, P, mode, pts, nrm=nrm)
    U, U0 = U.reshape(len(pts), W), U0.reshape(len(pts), W)
    for i in range(len(pts)):
        se = _se(U[i])
        assert abs(U[i].mean() - truth[i]) <= 4 * se + 2e-3, (i, U[i].mean(), truth[i], se)
    return U, U0


def test_neumann_data_2d_square():
    full, dir_, neu = wl.mixed_polygon([[-1, -1], [1, -1], [1, 1], [-1, 1]], [True, False, True, False],
                                       [16, 16, 16, 16], "square")
    od, on = orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(2, 1.0, 0.0)  # x^2 - y^2
    h = wl.Field(wl.FIELD_CONST, [], [-2.0])
    P = orc.walk_params(1e-3, 3000, 31)
    pts = np.array([[0.2, 0.3], [-0.6, -0.7], [0.5, 0.85]])
    truth = pts[:, 0] ** 2 - pts[:, 1] ** 2
    U, U0 = _check_neumann_data(od, on, g, h, P, pts, None, 1, truth)
    # the Neumann terms matter: without them the means are far off
    assert np.all(np.abs(U0.mean(1) - truth) > 20 * np.array([_se(u) for u in U0]))
    # from points on the Neumann side y = 1 (outward normal +y)
    f = np.array([[0.3, 1.0], [-0.8, 1.0]])
    _check_neumann_data(od, on, g, h, P, f, np.array([[0, 1.0]] * 2), 3, f[:, 0] ** 2 - 1)


def test_neumann_data_3d_box():
    _, od, on = _box([False, False, True, True, False, False])  # Neumann on y = +-1
    g = _sh(lambda x: x[:, 0] ** 2 - x[:, 1] ** 2)
    h = wl.Field(wl.FIELD_CONST, [], [-2.0])
    P = orc.walk_params(1e-3, 1500, 41)
    pts = np.array([[0.1, 0.5, -0.2], [-0.4, -0.8, 0.3]])
    truth = pts[:, 0] ** 2 - pts[:, 1] ** 2
    U, U0 = _check_neumann_data(od, on, g, h, P, pts, None, 1, truth)
    assert np.all(np.abs(U0.mean(1) - truth) > 20 * np.array([_se(u) for u in U0]))
    f = np.array([[0.3, -1.0, 0.2]])
    _check_neumann_data(od, on, g, h, P, f, np.array([[0, -1.0, 0]]), 3, f[:, 0] ** 2 - 1)


def test_box_first_ball_gradient():
    _, od, on = _box(TUBE)
    g = _sh(lambda x: x[:, 0], 1)
    eps, l = 1e-3, 5e-3
    W = 4000
    P = orc.walk_params(eps, W, 51)
    x = np.array([[1 - l, 0.2, -0.1], [1 - l, -0.5, 0.4]])
    n = np.array([[1.0, 0, 0]] * 2)
    xbar = x.copy()
    xbar[:, 0] = 1.0
    R0 = np.full(2, l)
    _, D, _ = orc.wost_walks(od, on, g, P, 0, x, nrm=n, R0=R0, xbar=xbar)
    D = D.reshape(2, W)
    for i in range(2):
        assert abs(D[i].mean() - 1.0) <= 4 * _se(D[i]) + 0.05
