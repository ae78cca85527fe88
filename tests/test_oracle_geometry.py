"""Pins of the oracle's geometry: closest points, inside tests, classification (not gpu)."""
import numpy as np
import pytest

import workloads as wl


def _random_polyline(rng, n):
    v = rng.normal(0, 1, (n, 2))
    p = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    return wl.Scene(2, v, p)


def _random_soup(rng, n):
    v = rng.normal(0, 1, (3 * n, 3))
    p = np.arange(3 * n).reshape(n, 3)
    return wl.Scene(3, v, p)


@pytest.mark.parametrize("dim,n", [(2, 5), (2, 64), (3, 7), (3, 64)])
def test_bvh_equals_brute_force(orc, dim, n):
    rng = np.random.default_rng(100 + n + dim)
    sc = _random_polyline(rng, n) if dim == 2 else _random_soup(rng, n)
    s = orc.Scene(sc)
    q = rng.normal(0, 1.5, (5000, dim))
    d1, x1, p1 = s.closest(q, brute=False)
    d2, x2, p2 = s.closest(q, brute=True)
    assert np.array_equal(d1, d2)
    assert np.array_equal(p1, p2)
    assert np.array_equal(x1, x2)


def test_point_segment_closed_forms(orc):
    sc = wl.Scene(2, np.array([[0.0, 0.0], [2.0, 0.0], [9, 9]]), np.array([[0, 1], [2, 2]]))
    # a degenerate far-away "segment" at (9,9) never wins
    s = orc.Scene(wl.Scene(2, np.array([[0.0, 0.0], [2.0, 0.0]]), np.array([[0, 1]])))
    d, xb, _ = s.closest(np.array([[0.5, 0.3], [-1.0, 1.0], [3.0, -4.0]]), brute=True)
    assert np.allclose(d, [0.3, np.sqrt(2), np.sqrt(1 + 16)], rtol=0, atol=1e-15)
    assert np.allclose(xb, [[0.5, 0], [0, 0], [2, 0]])
    del sc


def test_point_triangle_against_dense_sampling(orc):
    rng = np.random.default_rng(5)
    for _ in range(30):
        tri = rng.normal(0, 1, (3, 3))
        s = orc.Scene(wl.Scene(3, tri, np.array([[0, 1, 2]])))
        q = rng.normal(0, 1.5, (1, 3))
        d, xb, _ = s.closest(q, brute=True)
        m = 400
        a, b = np.meshgrid(np.linspace(0, 1, m), np.linspace(0, 1, m))
        keep = a + b <= 1
        bary = np.stack([1 - a[keep] - b[keep], a[keep], b[keep]], 1)
        pts = bary @ tri
        dd = np.linalg.norm(pts - q, axis=1).min()
        h = np.linalg.norm(tri[1:] - tri[0], axis=1).max() / (m - 1)
        assert d[0] <= dd + 1e-12
        assert d[0] >= dd - 2 * h
        # the reported point lies on the triangle plane and realises the distance
        nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        assert abs(np.dot(xb[0] - tri[0], nrm)) < 1e-12 * np.linalg.norm(nrm)
        assert abs(np.linalg.norm(xb[0] - q[0]) - d[0]) < 1e-13


def test_point_triangle_regions(orc):
    tri = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    s = orc.Scene(wl.Scene(3, tri, np.array([[0, 1, 2]])))
    q = np.array([[0.2, 0.2, 0.7], [-1, -1, 0.0], [2, -0.5, 0], [0.5, -1, 1], [1, 1, 0]])
    d, xb, _ = s.closest(q, brute=True)
    want = np.array([0.7, np.sqrt(2), np.sqrt(1 + 0.25), np.sqrt(2), np.sqrt(0.5)])
    assert np.allclose(d, want, atol=1e-15)
    assert np.allclose(xb[3], [0.5, 0, 0]) and np.allclose(xb[4], [0.5, 0.5, 0])


def test_winding_numbers(orc):
    circ = wl.circle_polygon(64)
    s = orc.Scene(circ)
    assert list(s.inside(np.array([[0.1, 0.2], [0.0, 0.0], [1.5, 0.0], [0.0, -2.0]]))) == [1, 1, 0, 0]
    # clockwise orientation gives -1, a doubly traversed circle gives 2
    cw = wl.Scene(2, circ.verts[::-1].copy(), circ.prims)
    assert orc.Scene(cw).inside(np.array([[0.1, 0.1]]))[0] == -1
    n = 64
    th = 4 * np.pi * np.arange(2 * n) / (2 * n)
    v = np.stack([np.cos(th), np.sin(th)], 1) * (1 + 0.01 * np.arange(2 * n)[:, None] / (2 * n))
    p = np.stack([np.arange(2 * n), (np.arange(2 * n) + 1) % (2 * n)], 1)
    assert orc.Scene(wl.Scene(2, v, p)).inside(np.array([[0.0, 0.1]]))[0] == 2


def test_3d_inside_by_pseudonormals(orc):
    sph = wl.icosphere(3)
    s = orc.Scene(sph)
    rng = np.random.default_rng(1)
    dirs = rng.normal(0, 1, (2000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = rng.uniform(0, 1.2, 2000)
    x = dirs * r[:, None]
    ins = s.inside(x)
    # the level-3 icosphere lies between radius cos(~4 deg) and 1
    sure_in = r < 0.99
    sure_out = r > 1.0 + 1e-9
    assert np.all(ins[sure_in] == 1)
    assert np.all(ins[sure_out] == 0)


def test_c1_grid_classification(orc):
    p = wl.problem_c1()
    s = orc.Scene(p.scene)
    cls = s.classify(p.eval_x, p.offset)
    inside_circle = (p.eval_x**2).sum(1) < 1
    # the polygon's sagitta (3e-4) is below the grid's clearance from the
    # circle (7.3e-4), so the inside sets agree
    assert np.array_equal(cls > 0, inside_circle)
    assert int((cls > 0).sum()) == 3228
    d, _, _ = s.closest(p.eval_x[cls > 0])
    assert np.array_equal(cls[cls > 0] == 2, d <= p.offset)
