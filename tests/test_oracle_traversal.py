"""Pins of the oracle's walk-query replay and BVH visit counter, the two
helpers behind the walk kernels' algorithmic traversal bytes.

- orc_walk_queries replays exactly the walk orc_walk takes (Section 3.1): as
  many queries as the walk's step count, the first at distance R0 from the
  start, the last one inside the epsilon shell or at the step cap.
- orc_bvh_visits counts a nearest-first query on the library's exported BVH;
  pinned against a separately written count in this file and against bounds
  that hold for any tree (a query visits at most every node and primitive, a
  hint that is already the closest primitive never adds work).
"""
import numpy as np
import pytest

import oracle
import workloads as wl


def _scene():
    return wl.star_polygon(256, 77, jitter="isotropic")


@pytest.fixture(scope="module")
def exported():
    from paper_2302_11825_amd import _bvc as B

    sc = _scene()
    h = B.bvc_scene_create(2, sc.verts, sc.prims)
    try:
        child, boxes, order = B.bvc_scene_export_bvh(h)
    finally:
        B.bvc_scene_destroy(h)
    return sc, child, boxes, order


def test_walk_queries_replay_the_walk():
    sc = _scene()
    osc = oracle.Scene(sc)
    c = osc.sample_cache(2000, 0.02, 2, 3)
    m = c["accept"]
    x, n, R0, xb = c["x"][m][:20], c["n"][m][:20], c["R0"][m][:20], c["xbar"][m][:20]
    P = oracle.walk_params(4e-3, 4, 9)
    g = wl.harmonic_2d(3, 1.0, 1.0)
    ids = np.arange(20) * 4 + 1
    q, h, own = oracle.walk_queries(osc, P, 0, x, R0, ids)
    for i in range(20):
        w = oracle.walk(osc, g, None, P, 0, x[i], n[i], R0[i], xb[i], int(ids[i]))
        qi = q[own == i]
        assert qi.shape[0] == w["steps"]
        assert abs(np.linalg.norm(qi[0] - x[i]) - R0[i]) <= 1e-12 * (1 + R0[i])
        d_last, _, _ = osc.closest(qi[-1:])
        assert d_last[0] < 4e-3 or qi.shape[0] == P.max_steps
        hi = h[own == i]
        assert hi[0] == -1 and np.all(hi[1:] >= 0)


def _seg_d2(x, a, b):
    # plain scalar arithmetic (no fused multiply-add, unlike a BLAS dot) and
    # exact endpoints when the projection clamps, so that ties at shared
    # vertices compare equal, as they must
    x0, x1, a0, a1, b0, b1 = (float(v) for v in (x[0], x[1], a[0], a[1], b[0], b[1]))
    e0, e1 = b0 - a0, b1 - a1
    t = ((x0 - a0) * e0 + (x1 - a1) * e1) / (e0 * e0 + e1 * e1)
    c0, c1 = (a0, a1) if t <= 0 else ((b0, b1) if t >= 1 else (a0 + t * e0, a1 + t * e1))
    return (x0 - c0) * (x0 - c0) + (x1 - c1) * (x1 - c1)


def _count(sc, child, boxes, order, x, hint):
    """Nearest-first count written out here: node 0 first; an entry is skipped
    when its box is farther than the best distance; the nearer child is taken
    first; leaves test their primitives in leaf order."""
    V, P = sc.verts, sc.prims
    d2p = lambda j: _seg_d2(x, V[P[j, 0]], V[P[j, 1]])
    best, nn, np_ = np.inf, 0, 0
    if hint >= 0:
        best, np_ = d2p(hint), 1
    todo = [(0, 0.0)]
    while todo:
        link, bound = todo.pop()
        if bound > best:
            continue
        if link < 0:
            s, k = (~link) >> 3, ((~link) & 7) + 1
            for j in range(s, s + k):
                np_ += 1
                best = min(best, d2p(order[j]))
            continue
        nn += 1
        bx = boxes[link].reshape(2, 2, 2)  # child, lo/hi, axis
        d = []
        for c in range(2):
            acc = 0.0
            for a in range(2):
                lo, hi, xa = float(bx[c, 0, a]), float(bx[c, 1, a]), float(x[a])
                e = lo - xa if xa < lo else (xa - hi if xa > hi else 0.0)
                acc += e * e
            d.append(acc)
        near = 1 if d[1] < d[0] else 0
        todo.append((child[link, 1 - near], d[1 - near]))
        todo.append((child[link, near], d[near]))
    return nn, np_


def test_bvh_visits_match_a_separate_count(exported):
    sc, child, boxes, order = exported
    osc = oracle.Scene(sc)
    rng = np.random.default_rng(12)
    q = rng.uniform(-1.3, 1.3, (60, 2))
    _, _, prim = osc.closest(q)
    hints = np.where(rng.random(60) < 0.5, prim, -1).astype(np.int32)
    vn, vp = oracle.bvh_visits(osc, child, boxes, order, q, hints)
    for i in range(60):
        assert (vn[i], vp[i]) == _count(sc, child, boxes, order, q[i], hints[i])


def test_bvh_visits_bounds(exported):
    sc, child, boxes, order = exported
    osc = oracle.Scene(sc)
    rng = np.random.default_rng(13)
    q = rng.uniform(-1.3, 1.3, (200, 2))
    _, _, prim = osc.closest(q)
    none = -np.ones(200, np.int32)
    vn0, vp0 = oracle.bvh_visits(osc, child, boxes, order, q, none)
    vn1, vp1 = oracle.bvh_visits(osc, child, boxes, order, q, prim)
    assert np.all(vn0 >= 1) and np.all(vn0 <= child.shape[0])
    assert np.all(vp0 >= 1) and np.all(vp0 <= sc.prims.shape[0])
    # the closest primitive as the hint never adds node work
    assert np.all(vn1 <= vn0)


@pytest.fixture(scope="module")
def exported3():
    from paper_2302_11825_amd import _bvc as B

    sc = wl.displaced_icosphere(2, 31)
    h = B.bvc_scene_create(3, sc.verts, sc.prims)
    try:
        child, boxes, order = B.bvc_scene_export_bvh(h)
        slabs = B.bvc_scene_export_slabs(h)
    finally:
        B.bvc_scene_destroy(h)
    return sc, child, boxes, order, slabs


def _subtree_prims(child, order, link):
    out, todo = [], [link]
    while todo:
        c = todo.pop()
        if c < 0:
            s, k = (~c) >> 3, ((~c) & 7) + 1
            out.extend(order[s:s + k])
        else:
            todo.extend(child[c])
    return np.array(out)


def test_slabs_hold_their_triangles(exported3):
    """Each child's slab axis is a unit vector and its range contains n.y for
    every vertex of every triangle below the child."""
    sc, child, boxes, order, slabs = exported3
    for node in range(child.shape[0]):
        for c in range(2):
            n, lo, hi = slabs[node, 5 * c:5 * c + 3], slabs[node, 5 * c + 3], slabs[node, 5 * c + 4]
            assert abs(np.linalg.norm(n) - 1.0) < 1e-14
            tri = _subtree_prims(child, order, child[node, c])
            s = sc.verts[sc.prims[tri].ravel()] @ n
            assert lo <= s.min() and s.max() <= hi
            assert s.min() - lo < 1e-12 and hi - s.max() < 1e-12
    assert np.all(slabs[:, 10:] == 0)


def test_slab_distance_bounds_the_subtree_distance(exported3):
    """The slab distance of a child never exceeds the distance from the point
    to the closest triangle below that child (brute force over the subtree)."""
    sc, child, boxes, order, slabs = exported3
    rng = np.random.default_rng(5)
    q = rng.uniform(-1.3, 1.3, (40, 3))
    for node in list(range(0, child.shape[0], 7)):
        for c in range(2):
            tri = _subtree_prims(child, order, child[node, c])
            sub = oracle.Scene(wl.Scene(3, sc.verts, np.ascontiguousarray(sc.prims[tri]), "sub"))
            d, _, _ = sub.closest(q, brute=True)
            n, lo, hi = slabs[node, 5 * c:5 * c + 3], slabs[node, 5 * c + 3], slabs[node, 5 * c + 4]
            t = q @ n
            e = np.maximum(np.maximum(lo - t, t - hi), 0.0)
            assert np.all(e <= d + 1e-12)


def test_slab_bounds_cut_work(exported3):
    """Pruning with the larger of the two bounds visits fewer nodes and
    primitives in total (not query by query: the nearer child can change, and
    with it the order in which the best distance falls)."""
    sc, child, boxes, order, slabs = exported3
    osc = oracle.Scene(sc)
    rng = np.random.default_rng(14)
    r = rng.uniform(0.2, 1.0, 300) ** (1 / 3)
    dvec = rng.normal(0, 1, (300, 3))
    q = dvec / np.linalg.norm(dvec, axis=1, keepdims=True) * r[:, None]
    _, _, prim = osc.closest(q)
    for hints in (-np.ones(300, np.int32), prim.astype(np.int32)):
        vn0, vp0 = oracle.bvh_visits(osc, child, boxes, order, q, hints)
        vn1, vp1 = oracle.bvh_visits(osc, child, boxes, order, q, hints, slabs=slabs)
        assert vn1.sum() < vn0.sum() and vp1.sum() < vp0.sum()
