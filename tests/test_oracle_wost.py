"""Pins of the oracle's walk on stars for mixed Dirichlet / Neumann
boundaries (the WoSt estimator of Section 3.1; 2D, h = 0, f = 0), against
facts independent of the oracle's arithmetic:

- with the Neumann part far away the walk is walk on spheres, walk by walk
  (same Philox streams as orc_walk);
- on the rectangle [0, 2] x [0, 1] with Dirichlet sides x = 0 (g = 0) and
  x = 2 (g = 2) and reflecting top and bottom, u = x: every walk ends on one
  of the two sides, so its mean is 2 P(exit right) = x within its standard
  error, from interior points and from points on the Neumann sides;
- a solution that varies along the Neumann sides, u = e^x cos y on
  [0, 1] x [0, pi] with Neumann sides y = 0 and y = pi (du/dn = 0 there);
- an L-shape with u = x (Neumann on the horizontal edges, Dirichlet on the
  vertical ones): the reflex corner is a Neumann/Dirichlet junction;
- the cache-walk gradient (mode 0) at offset Dirichlet points: n . grad u;
- the square [-1, 1]^2 without its fourth quadrant, Neumann on both edges of
  the 270 degree corner and u = r^(2/3) cos(2 phi/3) (zero normal derivative
  on both edges): the corner hides parts of balls centred in the first
  quadrant, so the silhouette bound on the star radius is what keeps the
  estimate unbiased.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl


def polygon_parts(verts, neumann):
    """Dirichlet and Neumann segment sets of the CCW polygon `verts`; segment
    i runs from vertex i to i + 1, Neumann where neumann[i]."""
    n = len(verts)
    segs = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.int32)
    V = np.asarray(verts, float)
    dir_ = wl.Scene(2, V, segs[~np.asarray(neumann)], "dirichlet")
    neu = wl.Scene(2, V, segs[np.asarray(neumann)], "neumann")
    full = wl.Scene(2, V, segs, "full")
    return full, dir_, neu


def subdivide(verts, neumann, k):
    """Each side split into k segments (flags copied)."""
    V, F = [], []
    n = len(verts)
    for i in range(n):
        a, b = np.asarray(verts[i], float), np.asarray(verts[(i + 1) % n], float)
        for j in range(k):
            V.append(a + (b - a) * j / k)
            F.append(neumann[i])
    return V, F


def _se(v):
    return v.std(ddof=1) / np.sqrt(v.size)


def test_wost_reduces_to_wos_without_neumann_nearby():
    scene = wl.circle_polygon(64)
    far = wl.Scene(2, np.array([[50.0, 50.0], [51.0, 50.0]]), np.array([[0, 1]], dtype=np.int32), "far")
    osc, ofar = orc.Scene(scene), orc.Scene(far)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    P = orc.walk_params(1e-3, 8, 5)
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.5, 0.5, (20, 2))
    U, _, st = orc.wost_walks(osc, ofar, g, P, 1, x)
    d, xb, _ = osc.closest(x)
    ref = np.array([orc.walk(osc, g, None, P, 1, x[i], None, d[i], xb[i], i * 8 + j)["U"]
                    for i in range(20) for j in range(8)])
    assert np.array_equal(U, ref)


def test_wost_rectangle_harmonic_measure():
    full, dir_, neu = polygon_parts(*subdivide([[0, 0], [2, 0], [2, 1], [0, 1]], [True, False, True, False], 8))
    od, on = orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(1, 1.0, 0.0)  # Re z = x
    W = 4000
    P = orc.walk_params(1e-4, W, 7)
    pts = np.array([[0.3, 0.5], [1.0, 0.2], [1.6, 0.85], [1.9, 0.5]])
    U, _, st = orc.wost_walks(od, on, g, P, 1, pts)
    U = U.reshape(len(pts), W)
    assert np.all((np.abs(U) < 1e-3) | (np.abs(U - 2) < 1e-3))  # exits on x = 0 or x = 2
    for i, x in enumerate(pts):
        assert abs(U[i].mean() - x[0]) < 5 * _se(U[i]) + 1e-3
    # from points on the Neumann sides (outward normals -y and +y)
    bpts = np.array([[0.7, 0.0], [1.4, 1.0]])
    nrm = np.array([[0.0, -1.0], [0.0, 1.0]])
    U3, _, _ = orc.wost_walks(od, on, g, P, 3, bpts, nrm=nrm)
    U3 = U3.reshape(2, W)
    for i, x in enumerate(bpts):
        assert abs(U3[i].mean() - x[0]) < 5 * _se(U3[i]) + 1e-3


def test_wost_solution_varying_along_neumann_sides():
    """u = e^x cos y on [0, 1] x [0, pi]: du/dn = -+e^x sin y = 0 on y = 0 and
    y = pi (Neumann), Dirichlet data on x = 0 and x = 1."""
    full, dir_, neu = polygon_parts(*subdivide([[0, 0], [1, 0], [1, np.pi], [0, np.pi]],
                                               [True, False, True, False], 16))
    od, on = orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(1, 0.0, 1.0)
    W = 3000
    P = orc.walk_params(1e-4, W, 9)
    pts = np.array([[0.5, 0.4], [0.3, 1.7], [0.8, 2.9], [0.5, 1.5707963]])
    U, _, _ = orc.wost_walks(od, on, g, P, 1, pts)
    U = U.reshape(len(pts), W)
    exact = wl.field_value(g, pts)
    for i in range(len(pts)):
        assert abs(U[i].mean() - exact[i]) < 5 * _se(U[i]) + 2e-3
    bpts = np.array([[0.35, 0.0], [0.7, np.pi]])
    U3, _, _ = orc.wost_walks(od, on, g, P, 3, bpts, nrm=np.array([[0.0, -1.0], [0.0, 1.0]]))
    U3 = U3.reshape(2, W)
    ex3 = wl.field_value(g, bpts)
    for i in range(2):
        assert abs(U3[i].mean() - ex3[i]) < 5 * _se(U3[i]) + 2e-3


def test_wost_l_shape_reflex_junction():
    """L-shape, u = x: Neumann on the horizontal edges (du/dn = 0), Dirichlet
    on the vertical ones; the reflex corner (1, 1) joins a Neumann and a
    Dirichlet edge."""
    verts = [[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]]
    neumann = [True, False, True, False, True, False]
    full, dir_, neu = polygon_parts(*subdivide(verts, neumann, 6))
    od, on = orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(1, 1.0, 0.0)
    W = 3000
    P = orc.walk_params(1e-4, W, 11)
    pts = np.array([[0.5, 0.5], [1.5, 0.5], [0.5, 1.5], [0.9, 0.9], [1.2, 0.95]])
    U, _, st = orc.wost_walks(od, on, g, P, 1, pts)
    U = U.reshape(len(pts), W)
    for i, x in enumerate(pts):
        assert abs(U[i].mean() - x[0]) < 5 * _se(U[i]) + 2e-3


def test_wost_cache_gradient():
    """Mode 0 at offset Dirichlet points of the rectangle with u = x: the
    normal derivative n . grad u = n_x (n from the point to the Dirichlet
    side)."""
    full, dir_, neu = polygon_parts(*subdivide([[0, 0], [2, 0], [2, 1], [0, 1]], [True, False, True, False], 8))
    ofull, od, on = orc.Scene(full), orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(1, 1.0, 0.0)
    l = 0.05
    x = np.array([[l, 0.5], [2 - l, 0.3]])
    nrm = np.array([[-1.0, 0.0], [1.0, 0.0]])
    R0, _, _ = ofull.closest(x)
    _, xb, _ = od.closest(x)
    W = 20000
    P = orc.walk_params(1e-4, W, 13)
    U, D, _ = orc.wost_walks(od, on, g, P, 0, x, nrm=nrm, R0=R0, xbar=xb)
    U, D = U.reshape(2, W), D.reshape(2, W)
    for i in range(2):
        assert abs(U[i].mean() - x[i, 0]) < 5 * _se(U[i]) + 1e-3
        assert abs(D[i].mean() - nrm[i, 0]) < 5 * _se(D[i]) + 0.02


@pytest.mark.parametrize("k", [1, 8])
def test_wost_reflex_neumann_corner(k):
    """k: segments per side (k = 1: the corner is the only Neumann vertex
    near the first quadrant, so nothing else bounds the star radius)."""
    verts = [[0, 0], [1, 0], [1, 1], [-1, 1], [-1, -1], [0, -1]]
    neumann = [True, False, False, False, False, True]
    full, dir_, neu = polygon_parts(*subdivide(verts, neumann, k))
    od, on = orc.Scene(dir_), orc.Scene(neu)
    g = wl.wedge_2d(1.0, 2.0 / 3.0)
    W = 6000
    P = orc.walk_params(1e-4, W, 17)
    pts = np.array([[0.3, 0.25], [0.2, 0.55], [0.6, 0.15], [-0.15, -0.4], [-0.4, 0.3]])
    U, _, _ = orc.wost_walks(od, on, g, P, 1, pts)
    U = U.reshape(len(pts), W)
    exact = wl.field_value(g, pts)
    for i in range(len(pts)):
        assert abs(U[i].mean() - exact[i]) < 5 * _se(U[i]) + 2e-3, (pts[i], U[i].mean(), exact[i], _se(U[i]))


def _inside_points(full, n, seed, margin=1e-3):
    of = orc.Scene(full)
    rng = np.random.default_rng(seed)
    lo, hi = full.bbox
    out = []
    while len(out) < n:
        x = rng.uniform(lo, hi, (4 * n, 2))
        d, _, _ = of.closest(x)
        out.extend(x[(of.inside(x) != 0) & (d > margin)])
    return np.array(out[:n])


def _nearest(x, verts):
    v = np.asarray(verts, float)
    return np.min(np.hypot(x[:, None, 0] - v[None, :, 0], x[:, None, 1] - v[None, :, 1]), axis=1)


def test_silhouette_distance_closed_forms():
    """The star radius's silhouette term by hand: straight wall vertices and
    convex corners are never silhouettes, run ends always are, and a reflex
    corner is one exactly for the viewpoints that see one of its edges hidden
    behind the other."""
    # rectangle, Neumann bottom and top: only the four run ends count, also
    # for walks standing on a wall
    full, _, neu = polygon_parts(*subdivide([[0, 0], [2, 0], [2, 1], [0, 1]], [True, False, True, False], 8))
    on = orc.Scene(neu)
    x = _inside_points(full, 300, 1)
    corners = [[0, 0], [2, 0], [2, 1], [0, 1]]
    assert np.allclose(orc.silhouette_distances(on, x), _nearest(x, corners), rtol=1e-15, atol=0)
    xw = np.stack([np.random.default_rng(2).uniform(0.05, 1.95, 40), np.repeat([0.0, 1.0], 20)], 1)
    assert np.allclose(orc.silhouette_distances(on, xw), _nearest(xw, corners), rtol=1e-15, atol=0)
    # a convex Neumann corner (2, 0) between the bottom and the right side
    full, _, neu = polygon_parts(*subdivide([[0, 0], [2, 0], [2, 1], [0, 1]], [True, True, False, False], 4))
    x = _inside_points(full, 300, 3)
    assert np.allclose(orc.silhouette_distances(orc.Scene(neu), x), _nearest(x, [[0, 0], [2, 1]]), rtol=1e-15,
                       atol=0)
    # the 270 degree corner at the origin between Neumann edges
    for k in (1, 8):
        full, _, neu = polygon_parts(*subdivide([[0, 0], [1, 0], [1, 1], [-1, 1], [-1, -1], [0, -1]],
                                                [True, False, False, False, False, True], k))
        x = _inside_points(full, 600, 4 + k)
        ends = _nearest(x, [[1, 0], [0, -1]])
        q1 = (x[:, 0] > 0) & (x[:, 1] > 0)
        q3 = (x[:, 0] < 0) & (x[:, 1] < 0)
        want = np.where(q1 | q3, np.minimum(ends, np.hypot(x[:, 0], x[:, 1])), ends)
        assert q1.sum() > 50 and q3.sum() > 50
        assert np.allclose(orc.silhouette_distances(orc.Scene(neu), x), want, rtol=1e-15, atol=0)
    # a thin Neumann cut (two runs folding back at the tip): the tip hides the
    # other side from every point, also from points on the cut's own line
    _, _, neu = wl.slit_disk_neumann(64, 16)
    x = np.array([[0.3, 0.0], [0.6, 0.0], [0.5, 0.2], [0.4, -0.3], [-0.5, 0.0]])
    ends = _nearest(x, [[1, 0]])
    want = np.minimum(ends, np.hypot(x[:, 0], x[:, 1]))
    assert np.allclose(orc.silhouette_distances(orc.Scene(neu), x), want, rtol=1e-15, atol=0)
