"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product path never imports
this package.  Arrays are numpy float64, row-major (n, dim).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


FLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall"]


def build(force: bool = True, path: str = LIB_PATH, native: bool = False) -> str:
    """Compile the oracle with gcc (plain C, FP64, no FMA contraction, no
    reassociation, so every flag set gives the same results).  The shared
    copy targets the generic x86-64 baseline, since it may run on another
    host than the one that built it; native=True adds -march=native for a
    copy built and timed on the same host (the CPU baseline)."""
    if force or not os.path.exists(path):
        flags = FLAGS + (["-march=native"] if native else [])
        cmd = ["gcc", *flags, "-o", path, os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
    return path


def load(path: str) -> None:
    """Use the oracle library at `path` from here on (e.g. a native build)."""
    global _lib, _lib_path
    _lib_path = path
    _lib = None
    lib()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_coef", C.c_int32), ("coef", _dp),
                ("param", C.c_double * 8)]


class _WalkParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_steps", C.c_int32), ("n_walks", C.c_int32),
                ("seed", C.c_uint64), ("batch", C.c_uint32), ("control_variate", C.c_int32),
                ("sigma", C.c_double), ("open_center", C.c_double * 3), ("open_radius", C.c_double),
                ("side_read", C.c_int32)]


_lib = None
_lib_path = LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build(path=_lib_path)
        L = C.CDLL(_lib_path)
        L.orc_scene_new.restype = C.c_void_p
        L.orc_scene_new.argtypes = [C.c_int, _dp, C.c_int64, _ip, C.c_int64]
        L.orc_scene_free.argtypes = [C.c_void_p]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_uniform_pair.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                       C.c_uint32, _dp, _dp]
        L.orc_closest_batch.argtypes = [C.c_void_p, C.c_int64, _dp, C.c_int, _dp, _dp, _ip]
        L.orc_inside.argtypes = [C.c_void_p, _dp]
        L.orc_inside.restype = C.c_int
        L.orc_classify.argtypes = [C.c_void_p, C.c_int64, _dp, C.c_double, _ip]
        L.orc_field_eval_batch.argtypes = [C.POINTER(_Field), C.c_int, C.c_int64, _dp, _dp]
        L.orc_basis_eval.argtypes = [C.POINTER(_Field), C.c_int, C.c_int, _dp]
        L.orc_basis_eval.restype = C.c_double
        L.orc_ein.argtypes = [C.c_double]
        L.orc_ein.restype = C.c_double
        L.orc_greens.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_sample_cache.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_int, C.c_uint64,
                                       C.c_uint32, _dp, _dp, _dp, _dp, _dp, _ip]
        L.orc_sample_cache.restype = C.c_int64
        L.orc_candidate_measure.argtypes = [C.c_void_p, C.c_double, C.c_int]
        L.orc_candidate_measure.restype = C.c_double
        L.orc_sample_sources.argtypes = [C.c_void_p, C.POINTER(_Field), C.c_int64, _dp, _dp,
                                         C.c_double, C.c_uint64, C.c_uint32, _dp, _dp]
        L.orc_walk.argtypes = [C.c_void_p, C.POINTER(_Field), C.POINTER(_Field),
                               C.POINTER(_WalkParams), C.c_int, _dp, _dp, C.c_double, _dp,
                               C.c_uint32, _dp, _dp, _dp, _dp, _ip, _ip]
        L.orc_cache_walks.argtypes = [C.c_void_p, C.POINTER(_Field), C.POINTER(_Field),
                                      C.POINTER(_WalkParams), C.c_int64, _dp, _dp, _dp, _dp,
                                      _dp, _dp, _dp, _dp, _ip]
        L.orc_cache_walks_subset.argtypes = [C.c_void_p, C.POINTER(_Field), C.POINTER(_Field),
                                             C.POINTER(_WalkParams), C.c_int64, _lp, _dp, _dp,
                                             _dp, _dp, _dp, _dp, _ip]
        L.orc_reduce.argtypes = [C.c_int64, C.c_int32, _dp, _dp, _dp, _dp]
        L.orc_pointwise.argtypes = [C.c_void_p, C.POINTER(_Field), C.POINTER(_Field),
                                    C.POINTER(_WalkParams), C.c_int64, _dp, _dp, _dp, _lp]
        L.orc_gather.argtypes = [C.c_int, C.c_int64, _dp, C.c_int64, _dp, _dp, _dp, _dp,
                                 C.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.orc_gather_backward.argtypes = [C.c_int, C.c_int64, _dp, _dp, C.c_int64, _dp, _dp, _dp,
                                          _dp, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_basis_means.argtypes = [C.POINTER(_Field), C.c_int, C.c_int64, C.c_int32, _dp, _dp,
                                      _dp, C.c_int, _dp, _dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_sample_direction.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                           C.c_uint32, C.c_int, _dp]
        L.orc_sample_ball_source.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                             C.c_uint32, C.c_int, _dp, C.c_double, _dp]
        L.orc_grad_radius.argtypes = [C.c_double]
        L.orc_grad_radius.restype = C.c_double
        L.orc_walk_queries.argtypes = [C.c_void_p, C.POINTER(_WalkParams), C.c_int, _dp, C.c_double,
                                       C.c_uint32, C.c_int32, _dp, _ip]
        L.orc_walk_queries.restype = C.c_int32
        L.orc_bvh_visits.argtypes = [C.c_void_p, C.c_int64, _ip, _dp, _dp, _ip, C.c_int64, _dp, _ip, _dp, _dp]
        for nm in ("orc_bessel_i0", "orc_bessel_i1", "orc_bessel_k0", "orc_bessel_k1"):
            getattr(L, nm).argtypes = [C.c_double]
            getattr(L, nm).restype = C.c_double
        L.orc_greens_sigma.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_screen_ball_weight.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_screen_ball_weight.restype = C.c_double
        L.orc_sample_grad_source.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, _dp,
                                             C.c_double, _dp, _dp, C.POINTER(C.c_double)]
        L.orc_sample_grad_source.restype = C.c_double
        L.orc_screen_grad_weight.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_screen_grad_weight.restype = C.c_double
        for nm in ("orc_screen_source_ratio", "orc_screen_grad_source_ratio"):
            getattr(L, nm).argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
            getattr(L, nm).restype = C.c_double
        L.orc_gather_sigma.argtypes = [C.c_int, C.c_double, C.c_int64, _dp, C.c_int64, _dp, _dp, _dp, _dp,
                                       C.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.orc_wost_walks.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(_Field), C.POINTER(_Field),
                                     C.POINTER(_WalkParams), C.c_int, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _ip]
        L.orc_silhouette_distances.argtypes = [C.c_void_p, C.c_int64, _dp, _dp]
        L.orc_silhouette_distances.restype = None
        L.orc_sphere_reentry.argtypes = [_dp, C.c_double, _dp, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_sphere_reentry.restype = C.c_int
        L.orc_sample_mixed.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                       C.c_uint64, C.c_uint32, _dp, _dp, _dp, _dp, _dp, _ip, _ip]
        L.orc_sample_mixed.restype = C.c_int64
        L.orc_sample_roi.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_uint32, _dp, _dp, _dp,
                                     _dp, _dp, _ip]
        L.orc_sample_roi.restype = C.c_int64
        L.orc_clamp_radius.argtypes = [C.c_int, C.c_double]
        L.orc_clamp_radius.restype = C.c_double
        L.orc_gather_clamped.argtypes = [C.c_int, C.c_int64, _dp, C.c_int64, _dp, _dp, _dp, _dp,
                                         C.c_int64, _dp, _dp, C.c_double, _dp]
        L.orc_offset_hits.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp, _dp, C.c_double, C.c_int32,
                                      _dp, _dp, _dp]
        L.orc_offset_hits.restype = C.c_int32
        L.orc_ray_direction.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, _dp]
        L.orc_clamp_correction.argtypes = [C.c_void_p, C.POINTER(_Field), C.POINTER(_Field),
                                           C.POINTER(_WalkParams), C.c_double, C.c_int, C.c_double, C.c_int32,
                                           C.c_int32, C.POINTER(_Field), C.c_int64, _dp, _dp, _lp]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _field(fld) -> _Field:
    F = _Field()
    if fld is None:
        F.kind = 0
        F.n_coef = 0
        F.coef = None
        return F
    F.kind = int(fld.kind)
    coef = _f64(fld.coef)
    F._keep = coef
    F.n_coef = int(coef.size)
    F.coef = coef.ctypes.data_as(_dp) if coef.size else None
    for i in range(8):
        F.param[i] = float(fld.param[i])
    return F


def num_threads() -> int:
    return lib().orc_num_threads()


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniform_pair(seed, block, id_, batch, tag):
    a = C.c_double()
    b = C.c_double()
    lib().orc_uniform_pair(seed, block, id_, batch, tag, C.byref(a), C.byref(b))
    return a.value, b.value


def ein(z: float) -> float:
    return lib().orc_ein(float(z))


def greens(dim, x, y, ny=None):
    x = _f64(x)
    y = _f64(y)
    ny = _f64(ny) if ny is not None else np.zeros(dim)
    G = np.zeros(1)
    dGdx = np.zeros(dim)
    dGdn = np.zeros(1)
    d2 = np.zeros(dim)
    lib().orc_greens(dim, _d(x), _d(y), _d(ny), _d(G), _d(dGdx), _d(dGdn), _d(d2))
    return G[0], dGdx, dGdn[0], d2


def field_eval(fld, x):
    x = _f64(x)
    out = np.zeros(x.shape[0])
    F = _field(fld)
    lib().orc_field_eval_batch(C.byref(F), x.shape[1], x.shape[0], _d(x), _d(out))
    return out


def basis_eval(fld, dim, m, x):
    x = _f64(x)
    F = _field(fld)
    return np.array([lib().orc_basis_eval(C.byref(F), dim, m, _d(np.ascontiguousarray(xi)))
                     for xi in x])


class Scene:
    """Oracle-side scene: copies the geometry and builds its own BVH."""

    def __init__(self, scene):
        self.dim = scene.dim
        v = _f64(scene.verts)
        p = np.ascontiguousarray(scene.prims, dtype=np.int32)
        self.h = lib().orc_scene_new(self.dim, _d(v), v.shape[0], _i(p), p.shape[0])

    def __del__(self):
        try:
            if self.h:
                lib().orc_scene_free(self.h)
        except Exception:
            pass

    def closest(self, x, brute=False):
        x = _f64(x).reshape(-1, self.dim)
        n = x.shape[0]
        d = np.zeros(n)
        xb = np.zeros((n, self.dim))
        pr = np.zeros(n, np.int32)
        lib().orc_closest_batch(self.h, n, _d(x), int(brute), _d(d), _d(xb), _i(pr))
        return d, xb, pr

    def inside(self, x):
        x = _f64(x).reshape(-1, self.dim)
        return np.array([lib().orc_inside(self.h, _d(np.ascontiguousarray(xi))) for xi in x])

    def classify(self, x, l):
        x = _f64(x).reshape(-1, self.dim)
        cls = np.zeros(x.shape[0], np.int32)
        lib().orc_classify(self.h, x.shape[0], _d(x), float(l), _i(cls))
        return cls

    def candidate_measure(self, l, sides):
        return lib().orc_candidate_measure(self.h, float(l), int(sides))

    def sample_cache(self, n, l, sides, seed, batch=0):
        d = self.dim
        x = np.zeros((n, d))
        nrm = np.zeros((n, d))
        w = np.zeros(n)
        xb = np.zeros((n, d))
        R0 = np.zeros(n)
        acc = np.zeros(n, np.int32)
        na = lib().orc_sample_cache(self.h, n, float(l), int(sides), int(seed), int(batch), _d(x),
                                    _d(nrm), _d(w), _d(xb), _d(R0), _i(acc))
        return dict(x=x, n=nrm, w=w, xbar=xb, R0=R0, accept=acc.astype(bool), n_accepted=na)

    def sample_sources(self, f, m, lo, hi, l, seed, batch=0):
        d = self.dim
        M = m**d
        y = np.zeros((M, d))
        sw = np.zeros(M)
        F = _field(f)
        lo = _f64(lo)
        hi = _f64(hi)
        lib().orc_sample_sources(self.h, C.byref(F), m, _d(lo), _d(hi), float(l), int(seed),
                                 int(batch), _d(y), _d(sw))
        return y, sw


def walk_params(eps, n_walks, seed, batch=0, max_steps=1024, control_variate=True, sigma=0.0, open_sphere=None,
                side_read=False):
    """open_sphere = (center, radius): an open 3D domain whose boundary the
    sphere encloses (Appendix B); walks outside it escape or re-enter.
    side_read: the side rule of double-sided data (Appendix B): exits and the
    control variate read g just off the boundary on the walk's side; off,
    they read it at the closest boundary point (Section 3.1)."""
    P = _WalkParams()
    P.side_read = int(bool(side_read))
    if open_sphere is not None:
        c, r = open_sphere
        for a in range(3):
            P.open_center[a] = float(c[a])
        P.open_radius = float(r)
    P.sigma = float(sigma)
    P.eps = float(eps)
    P.max_steps = int(max_steps)
    P.n_walks = int(n_walks)
    P.seed = int(seed)
    P.batch = int(batch)
    P.control_variate = int(bool(control_variate))
    return P


def walk(scene: Scene, g, f, params, mode, x, n, R0, xbar, id_):
    d = scene.dim
    x = _f64(x)
    n = _f64(n) if n is not None else None
    xbar = _f64(xbar)
    U = np.zeros(1)
    gr = np.zeros(d)
    ex = np.zeros(d)
    w1 = np.zeros(1)
    st = np.zeros(1, np.int32)
    cap = np.zeros(1, np.int32)
    G, Fv = _field(g), _field(f)
    lib().orc_walk(scene.h, C.byref(G), C.byref(Fv), C.byref(params), mode, _d(x), _d(n),
                   float(R0), _d(xbar), id_, _d(U), _d(gr), _d(ex), _d(w1), _i(st), _i(cap))
    return dict(U=U[0], grad=gr, exit=ex, w1=w1[0], steps=int(st[0]), capped=bool(cap[0]))


def walk_queries(scene: Scene, params, mode, x, R0, ids, max_q=None):
    """Query points (and hints: the previous query's closest primitive) of the
    walks `ids` started from x[i] with first radius R0[i], ids[i] the walk id
    (Section 3.1).  Returns (points [n, dim], hints [n], walk index [n])."""
    d = scene.dim
    max_q = int(max_q or params.max_steps)
    pts, hints, owner = [], [], []
    x = _f64(x).reshape(-1, d)
    for i, wid in enumerate(ids):
        q = np.zeros((max_q, d))
        h = np.zeros(max_q, np.int32)
        n = lib().orc_walk_queries(scene.h, C.byref(params), int(mode), _d(np.ascontiguousarray(x[i])),
                                   float(R0[i]), int(wid), max_q, _d(q), _i(h))
        pts.append(q[:n])
        hints.append(h[:n])
        owner.append(np.full(n, i))
    return np.concatenate(pts), np.concatenate(hints), np.concatenate(owner)


def bvh_visits(scene: Scene, child, boxes, order, q, hints, slabs=None):
    """Nodes expanded and primitive distances evaluated by a nearest-first
    query at each point q on the given BVH (child links, FP64 child boxes in
    the parent, leaf order, optional 3D slab bounds), seeded with the hint
    primitive."""
    child = np.ascontiguousarray(child, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    boxes = _f64(boxes)
    slabs = None if slabs is None else _f64(slabs)
    q = _f64(q).reshape(-1, scene.dim)
    hints = np.ascontiguousarray(hints, dtype=np.int32)
    nodes = np.zeros(q.shape[0])
    prims = np.zeros(q.shape[0])
    lib().orc_bvh_visits(scene.h, child.shape[0], _i(child), _d(boxes), _d(slabs), _i(order), q.shape[0],
                         _d(q), _i(hints), _d(nodes), _d(prims))
    return nodes, prims


def cache_walks(scene: Scene, g, f, params, cache, records=False):
    d = scene.dim
    x = _f64(cache["x"])
    n = x.shape[0]
    W = params.n_walks
    U = np.zeros(n * W)
    D = np.zeros(n * W)
    ex = np.zeros((n * W, d)) if records else None
    w1 = np.zeros(n * W) if records else None
    st = np.zeros(n * W, np.int32)
    G, Fv = _field(g), _field(f)
    lib().orc_cache_walks(scene.h, C.byref(G), C.byref(Fv), C.byref(params), n, _d(x),
                          _d(_f64(cache["n"])), _d(_f64(cache["R0"])), _d(_f64(cache["xbar"])),
                          _d(U), _d(D), _d(ex), _d(w1), _i(st))
    out = dict(U=U, D=D, steps=st)
    if records:
        out.update(exit=ex, w1=w1)
    return out


def cache_walks_subset(scene: Scene, g, f, params, cache, ids):
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    m = ids.size
    U = np.zeros(m)
    D = np.zeros(m)
    st = np.zeros(m, np.int32)
    G, Fv = _field(g), _field(f)
    lib().orc_cache_walks_subset(scene.h, C.byref(G), C.byref(Fv), C.byref(params), m,
                                 ids.ctypes.data_as(_lp), _d(_f64(cache["x"])),
                                 _d(_f64(cache["n"])), _d(_f64(cache["R0"])),
                                 _d(_f64(cache["xbar"])), _d(U), _d(D), _i(st))
    return dict(U=U, D=D, steps=st)


def reduce(U, D, W):
    U = _f64(U)
    D = _f64(D)
    n = U.size // W
    uh = np.zeros(n)
    dh = np.zeros(n)
    lib().orc_reduce(n, W, _d(U), _d(D), _d(uh), _d(dh))
    return uh, dh


def pointwise(scene: Scene, g, f, params, x, with_grad=True):
    x = _f64(x).reshape(-1, scene.dim)
    n = x.shape[0]
    u = np.zeros(n)
    gr = np.zeros((n, scene.dim)) if with_grad else None
    tot = C.c_int64()
    G, Fv = _field(g), _field(f)
    lib().orc_pointwise(scene.h, C.byref(G), C.byref(Fv), C.byref(params), n, _d(x), _d(u),
                        _d(gr), C.byref(tot))
    return u, gr, tot.value


def gather(dim, ex, cy, cn, a, b, sy=None, sw=None, with_grad=True, with_cond=False):
    ex = _f64(ex).reshape(-1, dim)
    cy = _f64(cy).reshape(-1, dim)
    cn = _f64(cn).reshape(-1, dim)
    a = _f64(a)
    b = _f64(b)
    K, N = ex.shape[0], cy.shape[0]
    if sy is None:
        sy = np.zeros((0, dim))
        sw = np.zeros(0)
    sy = _f64(sy).reshape(-1, dim)
    sw = _f64(sw)
    u = np.zeros(K)
    g = np.zeros((K, dim)) if with_grad else None
    c = np.zeros(K) if with_cond else None
    lib().orc_gather(dim, K, _d(ex), N, _d(cy), _d(cn), _d(a), _d(b), sy.shape[0], _d(sy),
                     _d(sw), _d(u), _d(g), _d(c))
    out = [u]
    if with_grad:
        out.append(g)
    if with_cond:
        out.append(c)
    return out[0] if len(out) == 1 else tuple(out)


def gather_backward(dim, ex, r, cy, cn, a, b, sy=None, sw=None):
    ex = _f64(ex).reshape(-1, dim)
    cy = _f64(cy).reshape(-1, dim)
    cn = _f64(cn).reshape(-1, dim)
    r = _f64(r)
    a = _f64(a)
    b = _f64(b)
    K, N = ex.shape[0], cy.shape[0]
    if sy is None:
        sy = np.zeros((0, dim))
        sw = np.zeros(0)
    sy = _f64(sy).reshape(-1, dim)
    sw = _f64(sw)
    M = sy.shape[0]
    da = np.zeros(N)
    db = np.zeros(N)
    ds = np.zeros(M)
    dx = np.zeros((K, dim))
    lib().orc_gather_backward(dim, K, _d(ex), _d(r), N, _d(cy), _d(cn), _d(a), _d(b), M, _d(sy),
                              _d(sw), _d(da), _d(db), _d(ds), _d(dx))
    return da, db, ds, dx


def basis_means(basis, dim, exit_pt, w1, xbar, W, cv=True):
    exit_pt = _f64(exit_pt).reshape(-1, dim)
    w1 = _f64(w1)
    xbar = _f64(xbar).reshape(-1, dim)
    n = xbar.shape[0]
    F = _field(basis)
    nb = F.n_coef if basis.kind != 3 else F.n_coef // (1 + dim)
    E = np.zeros((n, nb))
    Fm = np.zeros((n, nb))
    lib().orc_basis_means(C.byref(F), dim, n, W, _d(exit_pt), _d(w1), _d(xbar), int(cv), _d(E),
                          _d(Fm))
    return E, Fm


def sample_direction(seed, k, id_, batch, tag, dim):
    nu = np.zeros(dim)
    lib().orc_sample_direction(seed, k, id_, batch, tag, dim, _d(nu))
    return nu


def sample_grad_source(seed, id_, batch, tag, dim, c, R):
    """(t, yhat, y, m) of the first ball's gradient source sample."""
    yhat = np.zeros(dim)
    y = np.zeros(dim)
    m = C.c_double()
    t = lib().orc_sample_grad_source(seed, id_, batch, tag, dim, _d(_f64(c)), float(R), _d(yhat), _d(y),
                                     C.byref(m))
    return t, yhat, y, m.value


def sample_ball_source(seed, k, id_, batch, tag, dim, c, R):
    y = np.zeros(dim)
    lib().orc_sample_ball_source(seed, k, id_, batch, tag, dim, _d(_f64(c)), float(R), _d(y))
    return y


def grad_radius(u):
    return lib().orc_grad_radius(float(u))


# --- Clamped double-layer kernel and its bias correction (Section 3.3) ------
def clamp_radius(dim, c):
    """Distance beyond which |dG/dn| cannot exceed c."""
    return lib().orc_clamp_radius(int(dim), float(c))


def gather_clamped(dim, ex, cy, cn, a, b, c, sy=None, sw=None):
    """u with dG/dn clamped to [-c, c] in the boundary term (Eq. 9)."""
    ex = _f64(ex).reshape(-1, dim)
    cy = _f64(cy).reshape(-1, dim)
    cn = _f64(cn).reshape(-1, dim)
    a = _f64(a)
    b = _f64(b)
    if sy is None:
        sy = np.zeros((0, dim))
        sw = np.zeros(0)
    sy = _f64(sy).reshape(-1, dim)
    sw = _f64(sw)
    u = np.zeros(ex.shape[0])
    lib().orc_gather_clamped(dim, ex.shape[0], _d(ex), cy.shape[0], _d(cy), _d(cn), _d(a), _d(b), sy.shape[0],
                             _d(sy), _d(sw), float(c), _d(u))
    return u


def offset_hits(scene: Scene, l, sides, x, w, t_max, max_hits=64):
    """Crossings of the ray x + t w with the offset boundary, nearest first:
    (count, t, z, n) with at most max_hits rows."""
    d = scene.dim
    x = _f64(x).reshape(d)
    w = _f64(w).reshape(d)
    t = np.zeros(max_hits)
    z = np.zeros((max_hits, d))
    n = np.zeros((max_hits, d))
    cnt = lib().orc_offset_hits(scene.h, float(l), int(sides), _d(x), _d(w), float(t_max), int(max_hits), _d(t),
                                _d(z), _d(n))
    m = min(cnt, max_hits)
    return cnt, t[:m], z[:m], n[:m]


def ray_direction(seed, j, k, batch, dim):
    w = np.zeros(dim)
    lib().orc_ray_direction(int(seed), int(j), int(k), int(batch), int(dim), _d(w))
    return w


def clamp_correction(scene: Scene, g, f, params, l, sides, c, n_rays, max_hits, x, u_at_hits=None):
    """Second integral of Eq. 8 at the points x (inside the region the cache
    bounds): returns (corr, stats) with stats = (crossings, walks, rays with
    more than max_hits crossings)."""
    x = _f64(x).reshape(-1, scene.dim)
    n = x.shape[0]
    corr = np.zeros(n)
    st = np.zeros(3, np.int64)
    G, Fv = _field(g), _field(f)
    Uh = _field(u_at_hits) if u_at_hits is not None else None
    lib().orc_clamp_correction(scene.h, C.byref(G), C.byref(Fv), C.byref(params), float(l), int(sides), float(c),
                               int(n_rays), int(max_hits), C.byref(Uh) if Uh is not None else None, n, _d(x),
                               _d(corr), st.ctypes.data_as(_lp))
    return corr, st


# --- Screened Poisson (sigma > 0; Appendix A.2) -----------------------------
def bessel(name, x):
    """Modified Bessel function i0, i1, k0 or k1 of the oracle."""
    return getattr(lib(), "orc_bessel_" + name)(float(x))


def greens_sigma(dim, sigma, x, y, ny=None):
    x = _f64(x)
    y = _f64(y)
    ny = _f64(ny) if ny is not None else np.zeros(dim)
    G = np.zeros(1)
    dGdx = np.zeros(dim)
    dGdn = np.zeros(1)
    d2 = np.zeros(dim)
    lib().orc_greens_sigma(dim, float(sigma), _d(x), _d(y), _d(ny), _d(G), _d(dGdx), _d(dGdn), _d(d2))
    return G[0], dGdx, dGdn[0], d2


def screen_ball_weight(dim, sigma, R):
    return lib().orc_screen_ball_weight(int(dim), float(sigma), float(R))


def screen_grad_weight(dim, sigma, R):
    return lib().orc_screen_grad_weight(int(dim), float(sigma), float(R))


def screen_source_ratio(dim, sigma, R, t):
    return lib().orc_screen_source_ratio(int(dim), float(sigma), float(R), float(t))


def screen_grad_source_ratio(dim, sigma, R, t):
    return lib().orc_screen_grad_source_ratio(int(dim), float(sigma), float(R), float(t))


def gather_sigma(dim, sigma, ex, cy, cn, a, b, sy=None, sw=None, with_grad=True, with_cond=False):
    ex = _f64(ex).reshape(-1, dim)
    cy = _f64(cy).reshape(-1, dim)
    cn = _f64(cn).reshape(-1, dim)
    a = _f64(a)
    b = _f64(b)
    K, N = ex.shape[0], cy.shape[0]
    if sy is None:
        sy = np.zeros((0, dim))
        sw = np.zeros(0)
    sy = _f64(sy).reshape(-1, dim)
    sw = _f64(sw)
    u = np.zeros(K)
    g = np.zeros((K, dim)) if with_grad else None
    c = np.zeros(K) if with_cond else None
    lib().orc_gather_sigma(dim, float(sigma), K, _d(ex), N, _d(cy), _d(cn), _d(a), _d(b), sy.shape[0], _d(sy),
                           _d(sw), _d(u), _d(g), _d(c))
    out = [u]
    if with_grad:
        out.append(g)
    if with_cond:
        out.append(c)
    return out[0] if len(out) == 1 else tuple(out)


# --- Region of interest (Section 3.2, "Boundary Specification") ------------
def sample_roi(dom: Scene, roi: Scene, n, seed, batch=0):
    """Cache candidates on the boundary of the region `roi` inside `dom`."""
    d = roi.dim
    x = np.zeros((n, d))
    nrm = np.zeros((n, d))
    w = np.zeros(n)
    xb = np.zeros((n, d))
    R0 = np.zeros(n)
    acc = np.zeros(n, np.int32)
    na = lib().orc_sample_roi(dom.h, roi.h, n, int(seed), int(batch), _d(x), _d(nrm), _d(w), _d(xb), _d(R0), _i(acc))
    return dict(x=x, n=nrm, w=w, xbar=xb, R0=R0, accept=acc.astype(bool), n_accepted=na)


# --- Walk on stars, mixed Dirichlet / Neumann (2D, h = 0) --------------------
def wost_walks(dir_scene: Scene, neu_scene: Scene, g, params, mode, x, nrm=None, R0=None, xbar=None, h=None):
    """U (and D in mode 0) per walk, shape (n * W,); see orc_wost_walks.
    h: Neumann data (None: h = 0)."""
    d = dir_scene.dim
    x = _f64(x).reshape(-1, d)
    n, W = x.shape[0], params.n_walks
    U = np.zeros(n * W)
    D = np.zeros(n * W)
    st = np.zeros(n * W, np.int32)
    G = _field(g)
    H = _field(h)
    lib().orc_wost_walks(dir_scene.h, neu_scene.h, C.byref(G), C.byref(H), C.byref(params), int(mode), n, _d(x),
                         _d(_f64(nrm).reshape(-1, d)) if nrm is not None else None,
                         _d(_f64(R0)) if R0 is not None else None,
                         _d(_f64(xbar).reshape(-1, d)) if xbar is not None else None, _d(U), _d(D), _i(st))
    return U, D, st


def sample_mixed(full: Scene, dir_scene: Scene, neu_scene: Scene, n, l, seed, batch=0, junction_drop=0.0):
    """Cache candidates on the offset Dirichlet boundary and the Neumann part.
    junction_drop > 0 also rejects offset points closer than junction_drop * l
    to the Neumann part (0: the plain sampler)."""
    x = np.zeros((n, 2))
    nrm = np.zeros((n, 2))
    w = np.zeros(n)
    xb = np.zeros((n, 2))
    R0 = np.zeros(n)
    ty = np.zeros(n, np.int32)
    acc = np.zeros(n, np.int32)
    na = lib().orc_sample_mixed(full.h, dir_scene.h, neu_scene.h, n, float(l), float(junction_drop), int(seed),
                                int(batch), _d(x), _d(nrm),
                                _d(w), _d(xb), _d(R0), _i(ty), _i(acc))
    return dict(x=x, n=nrm, w=w, xbar=xb, R0=R0, type=ty, accept=acc.astype(bool), n_accepted=na)


def silhouette_distances(neu_scene: Scene, x):
    """Distance to the closest Neumann silhouette (2D vertex, 3D edge), per point."""
    x = _f64(x).reshape(-1, neu_scene.dim)
    d = np.zeros(x.shape[0])
    lib().orc_silhouette_distances(neu_scene.h, x.shape[0], _d(x), _d(d))
    return d


def sphere_reentry(center, radius, x, u, v, w):
    """orc_sphere_reentry for each row of x (n, 3) with uniforms u, v, w (n):
    returns (escaped (n,) bool, y (n, 3); NaN rows where escaped)."""
    L = lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    c = np.ascontiguousarray(center, dtype=np.float64)
    n = x.shape[0]
    esc = np.zeros(n, dtype=bool)
    y = np.full((n, 3), np.nan)
    yb = np.zeros(3)
    for i in range(n):
        e = L.orc_sphere_reentry(c.ctypes.data_as(_dp), float(radius), x[i].ctypes.data_as(_dp), float(u[i]),
                                 float(v[i]), float(w[i]), yb.ctypes.data_as(_dp))
        esc[i] = bool(e)
        if not e:
            y[i] = yb
    return esc, y
