"""Pins of double-sided Dirichlet boundaries (Appendix B, the Dirichlet part:
two sample sets, one on each offset side of a boundary curve that the domain
lies on both sides of), on the unit disk cut along [0, 1] x {0} with
u = r^(1/2) cos(phi/2), phi in [0, 2 pi) (sqrt(r) above the cut, -sqrt(r)
below it), against facts independent of the oracle's arithmetic:

- walks read the data on the side they reach the cut from: pointwise walk
  means match u within their standard errors just above and just below the
  cut (reading g on the wrong side would be off by 2 sqrt(r));
- the cache candidates on the cut's two offset sides are the lines y = +-l
  with normals towards the cut, and the round cap about the tip;
- Green's representation over the accepted samples with exact data
  reproduces u inside the offset region and vanishes in the band, across
  the jump of u;
- the whole chain (samples, walks, gather) estimates u.
"""
import numpy as np

import oracle as orc
import workloads as wl


def _grad_exact(x):
    """grad of Re sqrt(z) with the branch cut on the positive real axis."""
    r = np.hypot(x[:, 0], x[:, 1])
    phi = np.mod(np.arctan2(x[:, 1], x[:, 0]), 2 * np.pi)
    # f(z) = sqrt(r) e^{i phi/2}, f'(z) = 1 / (2 f): grad Re f = (Re f', -Im f')
    fp = 0.5 / (np.sqrt(r) * np.exp(0.5j * phi))
    return np.stack([fp.real, -fp.imag], 1)


def _se(v):
    return v.std(ddof=1) / np.sqrt(v.size)


def test_walks_read_the_side_they_reach():
    sc = wl.slit_disk(256, 64)
    osc = orc.Scene(sc)
    g = wl.slit_field()
    pts = np.array([[0.5, 0.02], [0.5, -0.02], [0.8, 0.004], [0.8, -0.004], [0.3, 0.3], [-0.4, -0.2],
                    [0.6, 0.0005], [0.6, -0.0005]])
    W = 3000
    P = orc.walk_params(1e-3, W, 5, side_read=True)
    d, xb, _ = osc.closest(pts)
    exact = wl.field_value(g, pts)
    for i, x in enumerate(pts):
        U = np.array([orc.walk(osc, g, None, P, 1, x, None, d[i], xb[i], i * W + j)["U"] for j in range(W)])
        assert abs(U.mean() - exact[i]) < 5 * _se(U) + 2e-3, (x, U.mean(), exact[i])
    # points inside the epsilon shell return g read from their own side
    sh = np.array([[0.5, 2e-4], [0.5, -2e-4]])
    d, xb, _ = osc.closest(sh)
    for i, x in enumerate(sh):
        u = orc.walk(osc, g, None, P, 1, x, None, d[i], xb[i], 0)["U"]
        assert abs(u - np.sign(x[1]) * np.sqrt(0.5)) < 1e-5
    # without the side rule both read g at the same closest point on the cut
    # (Section 3.1 as stated), so one of them gets the other side's value
    P0 = orc.walk_params(1e-3, W, 5)
    u0 = [orc.walk(osc, g, None, P0, 1, x, None, d[i], xb[i], 0)["U"] for i, x in enumerate(sh)]
    assert u0[0] == u0[1] and abs(abs(u0[0]) - np.sqrt(0.5)) < 1e-5


def test_double_sided_cache_samples():
    sc = wl.slit_disk(256, 64)
    osc = orc.Scene(sc)
    l, n = 0.05, 20000
    s = osc.sample_cache(n, l, 1, 9)
    acc = s["accept"]
    x, nv = s["x"][acc], s["n"][acc]
    near_cut = (x[:, 0] > 0) & (x[:, 0] < 0.8) & (np.abs(x[:, 1]) < 2 * l)
    up, dn = near_cut & (x[:, 1] > 0), near_cut & (x[:, 1] < 0)
    assert up.sum() > 100 and dn.sum() > 100 and abs(up.sum() - dn.sum()) < 0.2 * up.sum()
    assert np.allclose(x[up, 1], l, atol=1e-12) and np.allclose(x[dn, 1], -l, atol=1e-12)
    assert np.allclose(nv[up], [0, -1], atol=1e-12) and np.allclose(nv[dn], [0, 1], atol=1e-12)
    cap = (x[:, 0] < 0) & (np.hypot(x[:, 0], x[:, 1]) < 2 * l)
    assert cap.sum() > 10 and np.allclose(np.hypot(x[cap, 0], x[cap, 1]), l, atol=1e-12)
    # every accepted point is at distance l from the boundary and inside
    d, _, _ = osc.closest(x)
    assert np.allclose(d, l, rtol=1e-9) and np.all(osc.inside(x) != 0)


def test_green_representation_across_the_jump():
    sc = wl.slit_disk(256, 64)
    osc = orc.Scene(sc)
    l = 0.05
    s = osc.sample_cache(800000, l, 1, 3)  # about 49,000 accepted
    acc = s["accept"]
    z, nz, w = s["x"][acc], s["n"][acc], s["w"][acc]
    g = wl.slit_field()
    u = wl.field_value(g, z)
    dudn = np.sum(_grad_exact(z) * nz, 1)
    rng = np.random.default_rng(2)
    r = np.sqrt(rng.uniform(0.15**2, 0.85**2, 80))
    ph = rng.uniform(0.3, 2 * np.pi - 0.3, 80)
    xin = np.stack([r * np.cos(ph), r * np.sin(ph)], 1)
    got = orc.gather(2, xin, z, nz, u * w, dudn * w, with_grad=False)
    assert np.allclose(got, wl.field_value(g, xin), atol=1.5e-3)
    # inside the band about the cut the representation vanishes
    xb = np.stack([rng.uniform(0.2, 0.8, 20), rng.choice([-1, 1], 20) * rng.uniform(0.2, 0.6, 20) * l], 1)
    out = orc.gather(2, xb, z, nz, u * w, dudn * w, with_grad=False)
    assert np.all(np.abs(out) < 5e-3)


def test_double_sided_chain():
    sc = wl.slit_disk(256, 64)
    osc = orc.Scene(sc)
    g = wl.slit_field()
    l = 0.05
    s = osc.sample_cache(12000, l, 1, 13)  # about 750 accepted
    acc = s["accept"]
    cache = {k: s[k][acc] for k in ("x", "n", "w", "xbar", "R0")}
    W = 64
    ref = orc.cache_walks(osc, g, None, orc.walk_params(1e-3, W, 17, side_read=True), cache)
    uh, dh = orc.reduce(ref["U"], ref["D"], W)
    a, b = uh * cache["w"], dh * cache["w"]
    rng = np.random.default_rng(6)
    r = np.sqrt(rng.uniform(0.2**2, 0.8**2, 60))
    ph = rng.uniform(0.4, 2 * np.pi - 0.4, 60)
    x = np.stack([r * np.cos(ph), r * np.sin(ph)], 1)
    got = orc.gather(2, x, cache["x"], cache["n"], a, b, with_grad=False)
    ex = wl.field_value(g, x)
    assert np.sqrt(np.mean((got - ex) ** 2)) < 0.04 * np.sqrt(np.mean(ex**2))


def test_walk_on_stars_with_a_double_sided_neumann_cut():
    """u = r^(1/2) cos(phi/2) has zero flux through both sides of the cut, so
    with a reflecting cut and Dirichlet data on the circle it is the solution:
    walk-on-stars means match it just above and below the cut and from points
    on either side of the cut itself (a walk that crossed the cut, or reflected
    to the wrong side, would land near the other side's value)."""
    full, dir_, neu = wl.slit_disk_neumann(256, 64)
    od, on = orc.Scene(dir_), orc.Scene(neu)
    g = wl.slit_field()
    W = 3000
    P = orc.walk_params(1e-3, W, 31)
    pts = np.array([[0.5, 0.03], [0.5, -0.03], [0.2, 0.1], [0.2, -0.1], [-0.3, 0.2], [0.8, -0.02]])
    U, _, _ = orc.wost_walks(od, on, g, P, 1, pts)
    U = U.reshape(len(pts), W)
    ex = wl.field_value(g, pts)
    for i in range(len(pts)):
        assert abs(U[i].mean() - ex[i]) < 5 * _se(U[i]) + 2e-3, (pts[i], U[i].mean(), ex[i])
    # from the cut itself, on each side (outward normals point into the cut)
    bp = np.array([[0.4, 0.0], [0.4, 0.0], [0.7, 0.0], [0.7, 0.0]])
    nrm = np.array([[0.0, -1.0], [0.0, 1.0], [0.0, -1.0], [0.0, 1.0]])
    U3, _, _ = orc.wost_walks(od, on, g, P, 3, bp, nrm=nrm)
    U3 = U3.reshape(len(bp), W)
    want = np.array([1, -1, 1, -1]) * np.sqrt(bp[:, 0])
    for i in range(len(bp)):
        assert abs(U3[i].mean() - want[i]) < 5 * _se(U3[i]) + 2e-3, (bp[i], nrm[i], U3[i].mean(), want[i])
