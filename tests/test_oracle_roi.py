"""Pins of the oracle's region-of-interest cache (Section 3.2, "Boundary
Specification"; Algorithm 1 with p^dR = 1/|dR|):

- samples lie on the region's boundary, each in its own stratum of arc
  length (k + U_k)/n, with total weight |dR| and unit outward normals of R;
  distance and closest point come from the domain; samples outside the
  domain are rejected;
- the boundary integral over dR with exact data reproduces u inside R and
  vanishes outside it (Green's representation);
- the whole chain (samples, walks on the domain, gather) estimates the
  solution inside R and about zero outside.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl


def shifted(scene, scale, shift):
    return wl.Scene(scene.dim, scene.verts * scale + np.asarray(shift)[None], scene.prims, scene.name + "_roi")


def _arclength_positions(roi, x):
    """Position of each point along the CCW polygon, as a fraction of its length."""
    V, P = roi.verts, roi.prims
    a, b = V[P[:, 0]], V[P[:, 1]]
    L = np.linalg.norm(b - a, axis=1)
    cum = np.concatenate([[0.0], np.cumsum(L)])
    out = np.zeros(x.shape[0])
    for k, p in enumerate(x):
        t = np.sum((p - a) * (b - a), 1) / (L * L)
        res = np.linalg.norm(a + np.clip(t, 0, 1)[:, None] * (b - a) - p, axis=1)
        i = int(np.argmin(res))
        out[k] = (cum[i] + np.clip(t[i], 0, 1) * L[i]) / cum[-1]
    return out, cum[-1]


def test_roi_samples_2d():
    dom = wl.circle_polygon(256)
    roi = shifted(wl.circle_polygon(128), 0.4, (0.2, -0.1))
    odom, oroi = orc.Scene(dom), orc.Scene(roi)
    n = 3000
    s = orc.sample_roi(odom, oroi, n, 17, 2)
    assert s["accept"].all()
    d_roi, _, _ = oroi.closest(s["x"])
    assert np.all(d_roi < 1e-12)
    pos, perim = _arclength_positions(roi, s["x"])
    assert s["w"].sum() == pytest.approx(perim, rel=1e-12)
    k = np.arange(n)
    assert np.all(pos >= k / n - 1e-12) and np.all(pos <= (k + 1) / n + 1e-12)  # one point per stratum
    assert np.allclose(np.linalg.norm(s["n"], axis=1), 1.0)
    assert np.all(oroi.inside(s["x"] + 1e-6 * s["n"]) == 0) and np.all(oroi.inside(s["x"] - 1e-6 * s["n"]) != 0)
    d_dom, xb, _ = odom.closest(s["x"])
    assert np.allclose(s["R0"], d_dom, rtol=0, atol=1e-15)
    # xbar: the closest domain point
    assert np.allclose(s["xbar"], xb, atol=1e-15)
    # a region that leaves the domain: its outside samples are rejected
    roi2 = shifted(wl.circle_polygon(64), 0.5, (0.8, 0.0))
    s2 = orc.sample_roi(odom, orc.Scene(roi2), 2000, 3)
    inside = odom.inside(s2["x"]) != 0
    assert 0 < s2["n_accepted"] < 2000 and np.array_equal(s2["accept"], inside)


def test_roi_samples_3d():
    dom = wl.icosphere(3)
    roi = shifted(wl.icosphere(2), 0.45, (0.1, 0.05, -0.2))
    odom, oroi = orc.Scene(dom), orc.Scene(roi)
    s = orc.sample_roi(odom, oroi, 2000, 5)
    assert s["accept"].all()
    d_roi, _, _ = oroi.closest(s["x"])
    assert np.all(d_roi < 1e-12)
    V, P = roi.verts, roi.prims
    area = 0.5 * np.linalg.norm(np.cross(V[P[:, 1]] - V[P[:, 0]], V[P[:, 2]] - V[P[:, 0]]), axis=1).sum()
    assert s["w"].sum() == pytest.approx(area, rel=1e-12)
    assert np.all(oroi.inside(s["x"] + 1e-6 * s["n"]) == 0) and np.all(oroi.inside(s["x"] - 1e-6 * s["n"]) != 0)


def test_boundary_integral_vanishes_outside_the_region():
    """u(x) = int_dR [dG/dn u - G du/dn] for x in R, 0 for x outside R."""
    g = wl.harmonic_2d(3, 1.0, 1.0)
    c, rad, n = np.array([0.2, -0.1]), 0.4, 800
    t = 2 * np.pi * (np.arange(n) + 0.5) / n
    nv = np.stack([np.cos(t), np.sin(t)], 1)
    z = c[None] + rad * nv
    w = np.full(n, 2 * np.pi * rad / n)
    u = wl.field_value(g, z)
    dudn = np.sum(wl.field_grad_fd(g, z, 1e-6) * nv, 1)
    rng = np.random.default_rng(2)
    ang, rr = rng.uniform(0, 2 * np.pi, 30), rng.uniform(0, 0.7 * rad, 30)
    xin = c[None] + rr[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    rr2 = rng.uniform(1.3 * rad, 2.0 * rad, 30)
    xout = c[None] + rr2[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    uin = orc.gather(2, xin, z, nv, u * w, dudn * w, with_grad=False)
    uout = orc.gather(2, xout, z, nv, u * w, dudn * w, with_grad=False)
    assert np.allclose(uin, wl.field_value(g, xin), atol=1e-9)
    assert np.all(np.abs(uout) < 1e-9)


def test_roi_chain_estimates_the_solution():
    dom = wl.circle_polygon(256)
    roi = shifted(wl.circle_polygon(128), 0.4, (0.2, -0.1))
    odom, oroi = orc.Scene(dom), orc.Scene(roi)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    s = orc.sample_roi(odom, oroi, 1500, 23)
    W = 64
    P = orc.walk_params(1e-4, W, 31)
    cache = dict(x=s["x"], n=s["n"], w=s["w"], xbar=s["xbar"], R0=s["R0"])
    ref = orc.cache_walks(odom, g, None, P, cache)
    uh, dh = orc.reduce(ref["U"], ref["D"], W)
    a, b = uh * s["w"], dh * s["w"]
    rng = np.random.default_rng(4)
    ang = rng.uniform(0, 2 * np.pi, 40)
    c = np.array([0.2, -0.1])
    xin = c[None] + rng.uniform(0, 0.25, 40)[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    xout = c[None] + rng.uniform(0.55, 0.65, 40)[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
    uin = orc.gather(2, xin, s["x"], s["n"], a, b, with_grad=False)
    uout = orc.gather(2, xout, s["x"], s["n"], a, b, with_grad=False)
    err = np.sqrt(np.mean((uin - wl.field_value(g, xin)) ** 2))
    rms = np.sqrt(np.mean(wl.field_value(g, xin) ** 2))
    assert err < 0.02 * rms
    assert np.sqrt(np.mean(uout**2)) < 0.05 * rms
