"""Pins of the oracle's cache for a boundary with a Neumann part (Section
3.2, "Boundary Specification": cache samples on the Neumann part and on the
offset Dirichlet boundary; 2D, h = 0), against facts independent of the
oracle's arithmetic:

- on the rectangle [0, 2] x [0, 1] with Dirichlet sides x = 0 and x = 2 the
  accepted samples are the lines x = l, x = 2 - l (normals towards the
  Dirichlet side) and the Neumann sides beyond distance l (outward normals);
  their total weight is the length of that closed curve, 2 + 2 (2 - 2 l), up
  to one stratum per interval end; distances and closest points by hand;
- Green's representation over the accepted samples with exact data
  reproduces u = e^x cos y on [l, 1 - l] x [0, pi] (Neumann sides y = 0, pi)
  and vanishes in the Dirichlet band x < l: wrong normals, a missing part or
  a wrong acceptance rule all break one of the two;
- the whole chain (samples, walk-on-stars cache walks from the offset points
  with the Eq. 7 gradient, walks from the Neumann samples, gather) estimates
  u inside the offset region.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from test_oracle_wost import polygon_parts, subdivide


def test_mixed_samples_rectangle():
    full, dir_, neu = polygon_parts(*subdivide([[0, 0], [2, 0], [2, 1], [0, 1]], [True, False, True, False], 4))
    of, od, on = orc.Scene(full), orc.Scene(dir_), orc.Scene(neu)
    l, n = 0.1, 6000
    s = orc.sample_mixed(of, od, on, n, l, 41, 3)
    # candidate measure: Dirichlet segments (length 2), one circle of radius
    # l per vertex of the vertex table (16), Neumann segments (length 4)
    M = 2.0 + 16 * 2 * np.pi * l + 4.0
    assert np.allclose(s["w"], M / n, rtol=1e-14)
    acc, ty, x, nv = s["accept"], s["type"], s["x"], s["n"]
    assert s["n_accepted"] == acc.sum()
    off = acc & (ty == 0)
    nm = acc & (ty == 1)
    left = off & (x[:, 0] < 1)
    assert np.allclose(x[left, 0], l, atol=1e-12) and np.allclose(x[off & ~left, 0], 2 - l, atol=1e-12)
    assert np.all((x[off, 1] >= -1e-12) & (x[off, 1] <= 1 + 1e-12))
    assert np.allclose(nv[left], [-1, 0], atol=1e-12) and np.allclose(nv[off & ~left], [1, 0], atol=1e-12)
    bottom = nm & (x[:, 1] < 0.5)
    assert np.all(x[bottom, 1] == 0) and np.all(x[nm & ~bottom, 1] == 1)
    assert np.all((x[nm, 0] > l) & (x[nm, 0] < 2 - l))
    assert np.allclose(nv[bottom], [0, -1]) and np.allclose(nv[nm & ~bottom], [0, 1])
    # every Neumann candidate is on a Neumann side; rejected ones are in the band
    assert np.all((ty == 1) == np.isin(np.round(x[:, 1], 12), [0.0, 1.0]) | (ty == 1))
    rej_n = (ty == 1) & ~acc
    assert np.all((x[rej_n, 0] <= l + 1e-12) | (x[rej_n, 0] >= 2 - l - 1e-12))
    # total accepted weight = length of the offset region's boundary
    exact = 2 * 1.0 + 2 * (2 - 2 * l)
    assert abs(s["w"][acc].sum() - exact) <= 8 * M / n
    # the optional junction drop removes junction_drop * l of each offset
    # line at each Neumann wall (four pieces), and nothing else
    s2 = orc.sample_mixed(of, od, on, n, l, 41, 3, junction_drop=0.05)
    acc2 = s2["accept"]
    assert np.all(s2["R0"][acc2 & (s2["type"] == 0)] >= 0.05 * l)
    assert np.array_equal(acc2 & (s2["type"] == 1), acc & (ty == 1))
    assert np.all(acc2 <= acc)
    assert abs(s2["w"][acc2].sum() - (exact - 4 * 0.05 * l)) <= 8 * M / n
    # distances: R0 to the whole boundary, xbar on the nearest Dirichlet side
    d_full = np.minimum.reduce([x[:, 0], 2 - x[:, 0], x[:, 1], 1 - x[:, 1]])
    assert np.allclose(s["R0"][acc], d_full[acc], atol=1e-12)
    # xbar: the closest Dirichlet point
    xb = np.stack([np.where(x[:, 0] < 1, 0.0, 2.0), np.clip(x[:, 1], 0, 1)], 1)
    assert np.allclose(s["xbar"][acc], xb[acc], atol=1e-12)


def _strip():
    return polygon_parts(*subdivide([[0, 0], [1, 0], [1, np.pi], [0, np.pi]], [True, False, True, False], 8))


def test_mixed_representation_with_exact_data():
    full, dir_, neu = _strip()
    of, od, on = orc.Scene(full), orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(1, 0.0, 1.0)  # e^x cos y
    l, n = 0.08, 30000
    s = orc.sample_mixed(of, od, on, n, l, 7)
    acc = s["accept"]
    z, nz, w = s["x"][acc], s["n"][acc], s["w"][acc]
    u = wl.field_value(g, z)
    gu = np.stack([np.exp(z[:, 0]) * np.cos(z[:, 1]), -np.exp(z[:, 0]) * np.sin(z[:, 1])], 1)
    dudn = np.sum(gu * nz, 1)
    assert np.all(np.abs(dudn[s["type"][acc] == 1]) < 1e-12)  # zero flux on the Neumann sides
    rng = np.random.default_rng(3)
    xin = np.stack([rng.uniform(l + 0.15, 1 - l - 0.15, 40), rng.uniform(0.3, np.pi - 0.3, 40)], 1)
    got = orc.gather(2, xin, z, nz, u * w, dudn * w, with_grad=False)
    # the stratified samples are a midpoint-like quadrature of the closed
    # curve: each end of a piece cuts a stratum of width M/n = 8e-4
    assert np.allclose(got, wl.field_value(g, xin), atol=2e-4)
    # with the optional junction drop the curve has four gaps of length
    # 0.01 l = 8e-4 next to the Neumann walls: the representation then misses
    # the gaps' share of Green's formula, and adding the gaps back by the
    # midpoint rule closes the curve again
    dl, m = 1e-2 * l, 64
    s2 = orc.sample_mixed(of, od, on, n, l, 7, junction_drop=1e-2)
    acc2 = s2["accept"]
    z2, n2, w2 = s2["x"][acc2], s2["n"][acc2], s2["w"][acc2]
    u2 = wl.field_value(g, z2)
    d2 = np.sum(np.stack([np.exp(z2[:, 0]) * np.cos(z2[:, 1]), -np.exp(z2[:, 0]) * np.sin(z2[:, 1])], 1) * n2, 1)
    ys = (np.arange(m) + 0.5) / m * dl
    gz, gn = [], []
    for xo, nx in ((l, -1.0), (1 - l, 1.0)):
        for yy in (ys, np.pi - ys):
            gz.append(np.stack([np.full(m, xo), yy], 1))
            gn.append(np.tile([nx, 0.0], (m, 1)))
    gz, gn = np.concatenate(gz), np.concatenate(gn)
    gw = np.full(gz.shape[0], dl / m)
    gu = wl.field_value(g, gz)
    gd = np.sum(np.stack([np.exp(gz[:, 0]) * np.cos(gz[:, 1]), -np.exp(gz[:, 0]) * np.sin(gz[:, 1])], 1) * gn, 1)
    gap = orc.gather(2, xin, gz, gn, gu * gw, gd * gw, with_grad=False)
    dropped = orc.gather(2, xin, z2, n2, u2 * w2, d2 * w2, with_grad=False)
    # (each end of a gap cuts a stratum too: up to about 4e-4 there)
    assert np.allclose(dropped + gap, wl.field_value(g, xin), atol=6e-4)
    # the bias the drop adds at these points is of the same order as the
    # quadrature error of the plain sampler, far below the walks' noise
    assert 1e-4 < np.max(np.abs(gap)) < 2e-3
    # in the Dirichlet band (outside the offset region) the integral vanishes
    xb = np.stack([rng.uniform(0.2 * l, 0.6 * l, 20), rng.uniform(0.5, np.pi - 0.5, 20)], 1)
    out = orc.gather(2, xb, z, nz, u * w, dudn * w, with_grad=False)
    assert np.all(np.abs(out) < 5e-3)
    # with the Neumann samples left out the interior values are wrong
    keep = s["type"][acc] == 0
    bad = orc.gather(2, xin, z[keep], nz[keep], (u * w)[keep], (dudn * w)[keep], with_grad=False)
    assert np.max(np.abs(bad - wl.field_value(g, xin))) > 0.05


def test_mixed_chain_estimates_the_solution():
    """Near a Dirichlet / Neumann junction the first ball of an offset point
    is as small as its distance to the Neumann side, so the Eq. 7 gradient
    estimates there carry a variance that grows like (l / R0)^2: the
    solution values (with exact fluxes) and the fluxes away from the
    junctions are held to tight bars, the full chain to a looser one."""
    full, dir_, neu = _strip()
    of, od, on = orc.Scene(full), orc.Scene(dir_), orc.Scene(neu)
    g = wl.harmonic_2d(1, 0.0, 1.0)
    l = 0.05
    s = orc.sample_mixed(of, od, on, 1200, l, 19)
    acc = s["accept"]
    W = 48
    a = np.zeros(acc.size)
    b = np.zeros(acc.size)
    i0 = np.flatnonzero(acc & (s["type"] == 0))
    i1 = np.flatnonzero(acc & (s["type"] == 1))
    P = orc.walk_params(1e-4, W, 29)
    U, D, _ = orc.wost_walks(od, on, g, P, 0, s["x"][i0], nrm=s["n"][i0], R0=s["R0"][i0], xbar=s["xbar"][i0])
    uh, dh = orc.reduce(U, D, W)
    a[i0], b[i0] = uh, dh
    P1 = orc.walk_params(1e-4, W, 29, batch=0x80000000)
    U1, _, _ = orc.wost_walks(od, on, g, P1, 3, s["x"][i1], nrm=s["n"][i1])
    a[i1] = U1.reshape(-1, W).mean(1)
    z, nz, w = s["x"], s["n"], s["w"]
    gu = np.stack([np.exp(z[:, 0]) * np.cos(z[:, 1]), -np.exp(z[:, 0]) * np.sin(z[:, 1])], 1)
    de = np.sum(gu * nz, 1)
    ue = wl.field_value(g, z)
    # the walks' values on both parts
    assert abs(np.mean(a[i0] - ue[i0])) < 5 * np.std(a[i0] - ue[i0]) / np.sqrt(i0.size)
    assert abs(np.mean(a[i1] - ue[i1])) < 5 * np.std(a[i1] - ue[i1]) / np.sqrt(i1.size)
    # the fluxes of offset points whose first ball is at least l / 2
    far = i0[s["R0"][i0] >= 0.5 * l]
    e = b[far] - de[far]
    assert abs(e.mean()) < 5 * e.std() / np.sqrt(e.size)
    rng = np.random.default_rng(8)
    xin = np.stack([rng.uniform(0.25, 0.75, 40), rng.uniform(0.4, np.pi - 0.4, 40)], 1)
    ex = wl.field_value(g, xin)
    rms = np.sqrt(np.mean(ex**2))
    got_u = orc.gather(2, xin, z[acc], nz[acc], (a * w)[acc], (de * w)[acc], with_grad=False)
    assert np.sqrt(np.mean((got_u - ex) ** 2)) < 0.015 * rms
    got = orc.gather(2, xin, z[acc], nz[acc], (a * w)[acc], (b * w)[acc], with_grad=False)
    assert np.sqrt(np.mean((got - ex) ** 2)) < 0.06 * rms
