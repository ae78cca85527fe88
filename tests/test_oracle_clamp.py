"""Pins of the oracle's clamped double-layer kernel and its bias correction
(Section 3.3, Eqs. 8-9), against facts that do not come from the oracle's
own arithmetic:

- the clamped gather reduces to the plain gather as c grows without bound,
  and to the single-layer gather at c = 0 (Eq. 9's limits);
- every crossing the ray routine reports lies on the offset boundary
  {z inside : d(z) = l} (distance and inside test computed by the closest
  point and winding / pseudonormal routines, not by the ray routine);
- the signed crossings of any ray that starts inside the region {d > l} and
  leaves the scene sum to exactly 1 (each exit +1, each re-entry -1): a
  crossing missed, invented or with a flipped normal breaks the count, on a
  self-intersecting star (both offset sides), an L-shape with a reflex corner
  and displaced 3D spheres (edge cylinders and vertex spheres);
- on the L-shape the ray average of the weighted crossings equals the
  integral of dG/dn times the same weight over the offset boundary, taken by
  Gauss-Legendre quadrature along the offset boundary written out by hand
  (six straight pieces and the quarter circle around the reflex corner):
  the signed-solid-angle identity behind the correction;
- the correction with one walk per crossing matches the correction with the
  exact solution at the crossings within its Monte Carlo error.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl


def l_shape():
    verts = np.array([[0.0, 0.0], [2.0, 0.0], [2.0, 1.0], [1.0, 1.0], [1.0, 2.0], [0.0, 2.0]])
    prims = np.array([[i, (i + 1) % 6] for i in range(6)], dtype=np.int32)
    return wl.Scene(2, verts, prims, "l_shape")


def _points_in_region(osc, scene, l, n, rng, margin=0.0):
    lo, hi = scene.bbox
    out = []
    while len(out) < n:
        x = rng.uniform(lo, hi, (4 * n, scene.dim))
        d, _, _ = osc.closest(x)
        ok = (d > l * 1.05 + margin) & (osc.inside(x) != 0)
        out.extend(x[ok])
    return np.array(out[:n])


def _unit(rng, dim):
    v = rng.normal(0, 1, dim)
    return v / np.linalg.norm(v)


def test_clamped_gather_limits():
    rng = np.random.default_rng(1)
    for dim in (2, 3):
        N, K, M = 300, 40, 50
        cy = rng.normal(0, 1, (N, dim))
        cn = rng.normal(0, 1, (N, dim))
        cn /= np.linalg.norm(cn, axis=1, keepdims=True)
        a, b = rng.normal(0, 1, N), rng.normal(0, 1, N)
        sy, sw = rng.normal(0, 1, (M, dim)), rng.normal(0, 1, M)
        x = rng.normal(0, 0.5, (K, dim))
        u = orc.gather(dim, x, cy, cn, a, b, sy, sw, with_grad=False)
        assert np.array_equal(orc.gather_clamped(dim, x, cy, cn, a, b, 1e300, sy, sw), u)
        u0 = orc.gather(dim, x, cy, cn, np.zeros(N), b, sy, sw, with_grad=False)
        assert np.allclose(orc.gather_clamped(dim, x, cy, cn, a, b, 0.0, sy, sw), u0, rtol=1e-13, atol=1e-13)
        # in between, the clamp of Eq. 9 is odd: reversing every normal
        # (dG/dn -> -dG/dn) is the same as negating every a, once both signs
        # of dG/dn exceed c (checked below)
        c = 0.3 if dim == 2 else 0.03
        v1 = orc.gather_clamped(dim, x, cy, -cn, a, b, c, sy, sw)
        v2 = orc.gather_clamped(dim, x, cy, cn, -a, b, c, sy, sw)
        assert np.allclose(v1, v2, rtol=1e-13, atol=1e-13)
        Kn = np.array([[orc.greens(dim, x[k], cy[i], cn[i])[2] for i in range(N)] for k in range(K)])
        assert (Kn > c).sum() > 50 and (Kn < -c).sum() > 50
        # and it is a clamp: with every a_i = 1/N and no b or sources, u is the
        # mean of values in [-c, c] that equal dG/dn wherever |dG/dn| <= c
        u1 = orc.gather_clamped(dim, x, cy, cn, np.full(N, 1.0 / N), np.zeros(N), c)
        assert np.all(np.abs(u1) <= c * (1 + 1e-12))


SCENES_2D = [
    ("circle", lambda: wl.circle_polygon(97), 1, 0.05),
    ("star_selfintersecting", lambda: wl.star_polygon(512, 11, jitter="isotropic"), 2, 0.02),
    ("l_shape", l_shape, 1, 0.1),
]


def _scenes_3d():
    return [("displaced_icosphere", wl.displaced_icosphere(2, 5, amp=0.5), 1, 0.03)]


def _all_scenes():
    out = [(n, f(), s, l) for n, f, s, l in SCENES_2D]
    return out + _scenes_3d()


@pytest.mark.parametrize("case", range(4))
def test_crossings_lie_on_offset_boundary(case):
    name, scene, sides, l = _all_scenes()[case]
    osc = orc.Scene(scene)
    rng = np.random.default_rng(20 + case)
    xs = _points_in_region(osc, scene, l, 25, rng)
    total = 0
    for x in xs:
        for _ in range(8):
            w = _unit(rng, scene.dim)
            cnt, t, z, n = orc.offset_hits(osc, l, sides, x, w, 1e9)
            assert cnt == t.size
            total += cnt
            assert np.all(np.diff(t) >= 0)
            if cnt == 0:
                continue
            assert np.allclose(x + t[:, None] * w, z, atol=1e-12)
            d, xb, _ = osc.closest(z)
            assert np.all(np.abs(d - l) <= 1e-9 * l), name
            assert np.all(osc.inside(z) != 0)
            assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)
            # the normal points from z to its closest boundary point
            assert np.allclose(n, (xb - z) / l, atol=1e-6)
    assert total > 0


@pytest.mark.parametrize("case", range(4))
def test_signed_crossings_sum_to_one(case):
    name, scene, sides, l = _all_scenes()[case]
    osc = orc.Scene(scene)
    rng = np.random.default_rng(40 + case)
    xs = _points_in_region(osc, scene, l, 30, rng)
    multi = 0
    for x in xs:
        for _ in range(10):
            w = _unit(rng, scene.dim)
            cnt, t, z, n = orc.offset_hits(osc, l, sides, x, w, 1e9, max_hits=256)
            s = np.sign(n @ w)
            assert s.sum() == 1, (name, cnt, s)
            multi += cnt > 1
    if name != "circle":
        assert multi > 0  # some rays leave and re-enter the region


def _l_shape_offset_pieces(l):
    """The offset boundary of the L-shape at distance l, by hand: straight
    pieces (start, end, outward normal) and the quarter circle of radius l
    around the reflex corner (1, 1), angles from pi to 3 pi / 2."""
    segs = [
        ((l, l), (2 - l, l), (0, -1)),
        ((2 - l, l), (2 - l, 1 - l), (1, 0)),
        ((2 - l, 1 - l), (1, 1 - l), (0, 1)),
        ((1 - l, 1), (1 - l, 2 - l), (1, 0)),
        ((1 - l, 2 - l), (l, 2 - l), (0, 1)),
        ((l, 2 - l), (l, l), (-1, 0)),
    ]
    return [tuple(np.array(v, float) for v in s) for s in segs], (np.array([1.0, 1.0]), np.pi, 1.5 * np.pi)


def _boundary_integral(x, l, phi, panels=400, order=10):
    """Integral over the hand-written offset boundary of dG/dn(x, z) phi(z, K)."""
    gx, gw = np.polynomial.legendre.leggauss(order)
    segs, (cc, a0, a1) = _l_shape_offset_pieces(l)
    total = 0.0
    edges = np.linspace(0, 1, panels + 1)
    for p0, p1, nrm in segs:
        L = np.linalg.norm(p1 - p0)
        for a, b in zip(edges[:-1], edges[1:]):
            s = 0.5 * (a + b) + 0.5 * (b - a) * gx
            z = p0[None] + s[:, None] * (p1 - p0)[None]
            d = z - x
            K = (d @ nrm) / (2 * np.pi * np.sum(d * d, 1))
            total += np.sum(0.5 * (b - a) * gw * L * K * phi(z, K))
    for a, b in zip(edges[:-1], edges[1:]):
        s = 0.5 * (a + b) + 0.5 * (b - a) * gx
        ang = a0 + s * (a1 - a0)
        z = cc[None] + l * np.stack([np.cos(ang), np.sin(ang)], 1)
        nrm = (cc[None] - z) / l
        d = z - x
        K = np.sum(d * nrm, 1) / (2 * np.pi * np.sum(d * d, 1))
        total += np.sum(0.5 * (b - a) * gw * l * (a1 - a0) * K * phi(z, K))
    return total


def test_solid_angle_identity_on_the_l_shape():
    l = 0.1
    scene = l_shape()
    osc = orc.Scene(scene)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    uval = lambda z: wl.field_value(g, np.atleast_2d(z))
    S = 6000
    th = 2 * np.pi * (np.arange(S) + 0.5) / S
    dirs = np.stack([np.cos(th), np.sin(th)], 1)
    # near the reflex corner (rays meet the arc), near a straight piece, near
    # a corner where two straight pieces meet, and without clamping
    for x, c in (((0.93, 0.88), 2.0), ((1.5, 0.12), 5.0), ((0.125, 0.13), 3.0), ((0.93, 0.88), 0.0)):
        x = np.array(x)
        t_max = orc.clamp_radius(2, c)
        phi = lambda z, K: (np.maximum(0.0, 1 - c / np.abs(K)) if c > 0 else 1.0) * uval(z)
        acc = 0.0
        arc_hits = 0
        for w in dirs:
            cnt, t, z, n = orc.offset_hits(osc, l, 1, x, w, t_max)
            if cnt == 0:
                continue
            d = z - x
            K = np.sum(d * n, 1) / (2 * np.pi * np.sum(d * d, 1))
            acc += np.sum(np.sign(n @ w) * phi(z, K))
            arc_hits += int(np.sum(np.linalg.norm(z - np.array([1.0, 1.0]), axis=1) < l * (1 + 1e-9)))
        ray = acc / S
        quad = _boundary_integral(x, l, phi)
        assert abs(quad) > 1e-3
        assert abs(ray - quad) <= 1e-4 * abs(quad), (x, c, ray, quad)
        if x[1] > 0.5 and c > 0:  # the point by the reflex corner
            assert arc_hits > 0


def test_correction_walks_match_exact_values():
    """One walk per crossing (mode-1 walks, ids (k S + j) H + h) against the
    exact solution at the crossings on the same rays: the walk noise is the
    only difference, so the mean difference is zero within its error."""
    scene = wl.circle_polygon(128)
    osc = orc.Scene(scene)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    l, c = 0.05, 3.0
    rng = np.random.default_rng(9)
    ang = rng.uniform(0, 2 * np.pi, 40)
    rad = 1 - l - rng.uniform(0.005, 0.06, 40)
    x = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
    P = orc.walk_params(1e-4, 1, 77)
    corr_w, st = orc.clamp_correction(osc, g, None, P, l, 1, c, 32, 8, x)
    corr_e, st_e = orc.clamp_correction(osc, g, None, P, l, 1, c, 32, 8, x, u_at_hits=g)
    assert st[0] == st_e[0] and st[2] == 0 and st[1] > 100 and st_e[1] == 0
    diff = corr_w - corr_e
    # per point the walk noise is at most |weights| * (range of g) / S
    assert np.all(np.isfinite(diff))
    z = diff.mean() / (diff.std(ddof=1) / np.sqrt(diff.size))
    assert abs(z) < 4.5, z
    assert np.abs(corr_e).max() > 0.01  # the correction is not trivially zero here


def _l_shape_quadrature_cache(l, panels=600, order=10):
    """Gauss-Legendre nodes on the hand-written offset boundary of the
    L-shape: points, unit outward normals and arc-length weights."""
    gx, gw = np.polynomial.legendre.leggauss(order)
    segs, (cc, a0, a1) = _l_shape_offset_pieces(l)
    edges = np.linspace(0, 1, panels + 1)
    Z, N, Wt = [], [], []
    for p0, p1, nrm in segs:
        L = np.linalg.norm(p1 - p0)
        for a, b in zip(edges[:-1], edges[1:]):
            s = 0.5 * (a + b) + 0.5 * (b - a) * gx
            Z.append(p0[None] + s[:, None] * (p1 - p0)[None])
            N.append(np.repeat(nrm[None], order, 0))
            Wt.append(0.5 * (b - a) * gw * L)
    for a, b in zip(edges[:-1], edges[1:]):
        s = 0.5 * (a + b) + 0.5 * (b - a) * gx
        ang = a0 + s * (a1 - a0)
        z = cc[None] + l * np.stack([np.cos(ang), np.sin(ang)], 1)
        Z.append(z)
        N.append((cc[None] - z) / l)
        Wt.append(0.5 * (b - a) * gw * l * (a1 - a0))
    return np.concatenate(Z), np.concatenate(N), np.concatenate(Wt)


def test_eq8_reproduces_the_solution_on_the_l_shape():
    """Eq. 8 end to end with the exact boundary values: the clamped gather
    over an accurate quadrature of the offset boundary plus the ray-cast
    correction (exact u at the crossings) reproduces u(x) (Green's
    representation, Eq. 2), while the clamped gather alone is off by far
    more.  Pins the clamp (Eq. 9) and the correction's weights together."""
    l = 0.1
    scene = l_shape()
    osc = orc.Scene(scene)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    z, n, wq = _l_shape_quadrature_cache(l)
    gz = wl.field_value(g, z)
    dgdn = np.sum(wl.field_grad_fd(g, z, 1e-5) * n, 1)
    a, b = gz * wq, dgdn * wq
    for x, c in (((0.93, 0.88), 2.0), ((1.5, 0.12), 5.0), ((0.125, 0.13), 3.0)):
        x = np.array([x])
        exact = wl.field_value(g, x)[0]
        plain = orc.gather(2, x, z, n, a, b, with_grad=False)[0]
        assert abs(plain - exact) < 1e-6  # the quadrature cache is accurate
        clamped = orc.gather_clamped(2, x, z, n, a, b, c)[0]
        runs = []
        for sd in range(12):
            P = orc.walk_params(1e-4, 1, 1000 + sd)
            corr, st = orc.clamp_correction(osc, g, None, P, l, 1, c, 3000, 8, x, u_at_hits=g)
            assert st[2] == 0
            runs.append(corr[0])
        runs = np.array(runs)
        se = runs.std(ddof=1) / np.sqrt(runs.size)
        err = clamped + runs.mean() - exact
        assert abs(err) <= 4.5 * se + 1e-6, (x, c, err, se)
        assert abs(clamped - exact) > 5 * (4.5 * se + 1e-6)  # the clamp alone is biased


def test_correction_recomposed_from_single_walks():
    """orc_clamp_correction equals its definition assembled from the single
    routines: ray j of point k from the tag-5 direction, its crossings, and
    one mode-1 walk from each contributing crossing (|dG/dn| > c, rank h
    among them, nearest first) with id (k S + j) H + h."""
    # a jagged self-intersecting star: rays often meet several crossings
    scene = wl.star_polygon(256, 5, jitter="isotropic")
    osc = orc.Scene(scene)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    l, c, S, H, sides = 0.01, 0.5, 6, 4, 2
    x = _points_in_region(osc, scene, l, 40, np.random.default_rng(3))
    d0, _, _ = osc.closest(x)
    x = x[np.argsort(d0)[:4]]  # the four nearest the boundary
    P = orc.walk_params(1e-4, 1, 4242, batch=3)
    corr, st = orc.clamp_correction(osc, g, None, P, l, sides, c, S, H, x)
    t_max = orc.clamp_radius(2, c)
    walks, later = 0, 0
    for k in range(x.shape[0]):
        acc = 0.0
        for j in range(S):
            w = orc.ray_direction(4242, j, k, 3, 2)
            cnt, t, z, n = orc.offset_hits(osc, l, sides, x[k], w, t_max, 256)
            h = 0
            for i in range(cnt):
                K = orc.greens(2, x[k], z[i], n[i])[2]
                if abs(K) <= c or h >= H:
                    continue
                d, xb, _ = osc.closest(z[i])
                U = orc.walk(osc, g, None, P, 1, z[i], None, d[0], xb[0], (k * S + j) * H + h)["U"]
                acc += np.sign(K) * (1 - c / abs(K)) * U
                walks += 1
                later += h > 0
                h += 1
        assert corr[k] == pytest.approx(acc / S, rel=1e-12, abs=1e-14)
    assert walks == st[1] and later > 0


def test_ray_direction_convention():
    """Ray j of point k: angle 2 pi ua (2D) or z = 1 - 2 ua, phi = 2 pi ub
    (3D) from the Philox pair of block j, id k, tag 5."""
    for j, k in ((0, 0), (3, 17), (1000, 123456)):
        ua, ub = orc.uniform_pair(99, j, k, 2, 5)
        w2 = orc.ray_direction(99, j, k, 2, 2)
        assert np.allclose(w2, [np.cos(2 * np.pi * ua), np.sin(2 * np.pi * ua)], atol=1e-15)
        w3 = orc.ray_direction(99, j, k, 2, 3)
        zz = 1 - 2 * ua
        rho = np.sqrt(max(0.0, 1 - zz * zz))
        assert np.allclose(w3, [rho * np.cos(2 * np.pi * ub), rho * np.sin(2 * np.pi * ub), zz], atol=1e-15)
