"""Boundary Value Caching on one GPU: Algorithm 1 (UpdateSolution) as a
sequence of C-ABI calls.

    cache points on the offset boundary   bvc_sample_cache + bvc_compact + bvc_take
    walks from every cache point          bvc_cache_walks            (Section 3.1, Eq. 7)
    cache means  u-hat, du/dn-hat         bvc_reduce_walks
    source samples                        bvc_sample_sources         (Eq. 4)
    interior / band classification        bvc_classify + bvc_compact (Section 3.2)
    gather of u and grad u                bvc_gather_u / _grad       (Eqs. 3-6)
    pointwise walks for band points       bvc_pointwise_wos          (Section 3.2)

This module only allocates device memory (torch) and sequences calls; every
step runs in the library's kernels on torch's current stream.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _bvc as B

DT = {"f32": torch.float32, "f64": torch.float64}
CODE = {"f32": B.F32, "f64": B.F64}


class DeviceField:
    """A field descriptor with its coefficients resident on the device."""

    def __init__(self, fld, device="cuda"):
        self.kind = int(fld.kind)
        self.param = [float(v) for v in fld.param]
        coef = np.ascontiguousarray(fld.coef, dtype=np.float64)
        self.coef = torch.from_numpy(coef).to(device) if coef.size else None

    def c(self) -> B.bvc_field:
        return B.make_field(self.kind, self.coef, self.param)


class Scene:
    """Host BVH build and upload into a torch-owned device buffer."""

    def __init__(self, scene, device="cuda"):
        self.dim = scene.dim
        self.h = B.bvc_scene_create(scene.dim, scene.verts, scene.prims)
        info = B.bvc_scene_get_info(self.h)
        self.buf = torch.empty(int(info.device_bytes), dtype=torch.uint8, device=device)
        B.bvc_scene_upload(self.h, self.buf)
        self.info = B.bvc_scene_get_info(self.h)
        self.device = device
        self._scratch = {}

    def __del__(self):
        try:
            B.bvc_scene_destroy(self.h)
        except Exception:
            pass

    @property
    def lo(self):
        return list(self.info.lo)[: self.dim]

    @property
    def hi(self):
        return list(self.info.hi)[: self.dim]

    def scratch_int(self, n):
        k = ("compact", n)
        if k not in self._scratch:
            self._scratch[k] = torch.empty(B.bvc_compact_scratch_ints(n), dtype=torch.int32, device=self.device)
        return self._scratch[k]

    def order_work(self):
        k = ("order",)
        if k not in self._scratch:
            self._scratch[k] = torch.empty(B.bvc_spatial_order_workspace_bytes(), dtype=torch.uint8,
                                           device=self.device)
        return self._scratch[k]

    @property
    def ordered_walks(self) -> bool:
        """Whether walks start in spatial order: when the FP32 traversal data
        (nodes with their slab bounds, primitives) exceed one XCD's 4 MiB L2,
        walks in flight together should query one part of the tree.  Smaller
        trees stay in L2 whatever the order, and there the order's
        indirection only costs."""
        i = self.info
        node, prim = (48, 16) if self.dim == 2 else (104, 48)
        return i.n_nodes * node + i.n_prims * prim > (4 << 20)

    def spatial_order(self, x, n, n_dev=None):
        """Launch order of the points x ([dim][ld], ld >= n) by position, for
        the walks' `order` (bvc_spatial_order): walks started together then
        query nearby parts of the tree.  Results do not depend on it."""
        order = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        B.bvc_spatial_order(self.h, n, x, order, self.order_work(), n_dev=n_dev)
        return order

    def compact(self, flags, want):
        n = flags.numel()
        idx = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        cnt = B.bvc_compact(n, flags, want, idx, self.scratch_int(n))
        return idx, cnt


class Cache:
    """Accepted cache samples, FP64: x, nrm, xbar [d][cap], w, R0 [cap].

    A cache compacted with its count read back holds n = cap points.  One
    sampled without the readback (sample_cache_device) keeps the count on the
    device (n_dev, int64 [1]) and cap entries of room; the calls that consume
    it read the count there, and reading `n` on the host synchronises."""

    def __init__(self, n, x, nrm, w, xbar, R0, n_candidates=0, n_dev=None, cap=None):
        self._n = n
        self.x, self.nrm, self.w, self.xbar, self.R0 = x, nrm, w, xbar, R0
        self.n_candidates = n_candidates
        self.n_dev = n_dev
        self.cap = n if cap is None else cap
        self.order = None  # launch order of the walks, made by cache_walks

    @property
    def n(self) -> int:
        if self._n is None:
            raw = int(self.n_dev[0].item())
            if raw > self.cap:
                raise RuntimeError(f"cache overflow: {raw} accepted candidates for a capacity of {self.cap}; the "
                                   f"step used the first {self.cap} (raise cache_cap)")
            self._n = raw
        return self._n


def take(src, idx, n, rows, ld_in, dtype_out=torch.float64, count=None):
    """Columns idx[0..n) of src (all columns when idx is None) as [rows][n];
    with a device count, the first min(n, count) only (n is the capacity)."""
    out = torch.empty((rows, max(n, 1)) if rows > 1 else (max(n, 1),), dtype=dtype_out, device=src.device)
    if count is None:
        B.bvc_take(B.dtype_code(src.dtype), B.dtype_code(dtype_out), n, idx, rows, ld_in, src, max(n, 1), out)
    else:
        B.bvc_take_count(B.dtype_code(src.dtype), B.dtype_code(dtype_out), n, count, idx, rows, ld_in, src,
                         max(n, 1), out)
    return out


def sample_cache(sc: Scene, n_cand, l, sides, seed, batch=0) -> Cache:
    d, dev = sc.dim, sc.device
    f64 = torch.float64
    x = torch.empty(d, n_cand, dtype=f64, device=dev)
    nrm = torch.empty_like(x)
    xbar = torch.empty_like(x)
    w = torch.empty(n_cand, dtype=f64, device=dev)
    R0 = torch.empty_like(w)
    acc = torch.empty(n_cand, dtype=torch.int32, device=dev)
    B.bvc_sample_cache(sc.h, n_cand, l, sides, seed, batch, x, nrm, w, xbar, R0, acc)
    idx, n = sc.compact(acc, 1)
    c = Cache(n, take(x, idx, n, d, n_cand), take(nrm, idx, n, d, n_cand), take(w, idx, n, 1, n_cand),
              take(xbar, idx, n, d, n_cand), take(R0, idx, n, 1, n_cand), n_cand)
    return c


def sample_cache_device(sc: Scene, n_cand, cap, l, sides, seed, batch=0) -> Cache:
    """sample_cache without the count readback: the accepted count stays on
    the device and the compacted arrays have room for `cap` points (the
    first cap accepted candidates are kept; Cache.n reports an overflow)."""
    d, dev = sc.dim, sc.device
    f64 = torch.float64
    x = torch.empty(d, n_cand, dtype=f64, device=dev)
    nrm = torch.empty_like(x)
    xbar = torch.empty_like(x)
    w = torch.empty(n_cand, dtype=f64, device=dev)
    R0 = torch.empty_like(w)
    acc = torch.empty(n_cand, dtype=torch.int32, device=dev)
    B.bvc_sample_cache(sc.h, n_cand, l, sides, seed, batch, x, nrm, w, xbar, R0, acc)
    idx = torch.empty(max(n_cand, 1), dtype=torch.int32, device=dev)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    B.bvc_compact_count(n_cand, acc, 1, idx, sc.scratch_int(n_cand), count)
    return Cache(None, take(x, idx, cap, d, n_cand, count=count), take(nrm, idx, cap, d, n_cand, count=count),
                 take(w, idx, cap, 1, n_cand, count=count), take(xbar, idx, cap, d, n_cand, count=count),
                 take(R0, idx, cap, 1, n_cand, count=count), n_cand, n_dev=count, cap=cap)


def sample_roi(dom: Scene, roi: Scene, n_cand, seed, batch=0) -> Cache:
    """Cache points on the boundary of a region of interest inside the domain
    (Section 3.2), compacted to the accepted ones."""
    d, dev = dom.dim, dom.device
    f64 = torch.float64
    x = torch.empty(d, n_cand, dtype=f64, device=dev)
    nrm = torch.empty_like(x)
    xbar = torch.empty_like(x)
    w = torch.empty(n_cand, dtype=f64, device=dev)
    R0 = torch.empty_like(w)
    acc = torch.empty(n_cand, dtype=torch.int32, device=dev)
    B.bvc_sample_roi(dom.h, roi.h, n_cand, seed, batch, x, nrm, w, xbar, R0, acc)
    idx, n = dom.compact(acc, 1)
    return Cache(n, take(x, idx, n, d, n_cand), take(nrm, idx, n, d, n_cand), take(w, idx, n, 1, n_cand),
                 take(xbar, idx, n, d, n_cand), take(R0, idx, n, 1, n_cand), n_cand)


def candidates_for(sc: Scene, n_target, l, sides, seed, pilot=65536):
    """Number of candidates whose expected accepted count is n_target, from a
    pilot draw with an independent batch index."""
    c = sample_cache(sc, pilot, l, sides, seed, batch=0x7FFFFFFF)
    rate = max(c.n, 1) / pilot
    return int(math.ceil(n_target / rate))


def walk_params(eps, n_walks, seed, g: DeviceField, f: Optional[DeviceField], dtype="f32", batch=0,
                max_steps=1024, control_variate=True, blocks=0, sigma=0.0, open_sphere=None,
                side_read=False, h: Optional[DeviceField] = None) -> B.bvc_walk_params:
    """open_sphere = (centre, radius) of a sphere enclosing the scene: an open
    3D domain (Appendix B), whose walks escape to infinity or re-enter.
    side_read: the side rule of double-sided data (Appendix B); off, walks
    read g at the closest boundary point (Section 3.1).  h: Neumann data of
    the walk on stars (None: h = 0)."""
    p = B.bvc_walk_params()
    p.side_read = int(bool(side_read))
    p.sigma = float(sigma)
    if open_sphere is not None:
        c, r = open_sphere
        for a in range(3):
            p.open_center[a] = float(c[a])
        p.open_radius = float(r)
    p.eps = float(eps)
    p.max_steps = int(max_steps)
    p.n_walks = int(n_walks)
    p.seed = int(seed)
    p.batch = int(batch)
    p.control_variate = int(bool(control_variate))
    p.dtype = CODE[dtype]
    p.blocks = int(blocks)
    p.g = g.c()
    p.f = f.c() if f is not None else B.make_field(0, None, [])
    p.h = h.c() if h is not None else B.make_field(0, None, [])
    # the struct holds raw device pointers to the fields' coefficients: keep
    # the fields alive as long as the struct is
    p._fields_keep = (g, f, h)
    return p


def cache_walks(sc: Scene, cache: Cache, params: B.bvc_walk_params, dtype="f32", records=False, started=None):
    """Walks from every cache point; a cache with a device count is walked up
    to that count (outputs laid out for its capacity).  started: an event
    recorded on the stream right before the walk launch, or None."""
    dev = sc.device
    n, W = cache.cap, params.n_walks
    if cache.n_dev is not None:
        params.n_dev = cache.n_dev.data_ptr()
    _set_cache_order(sc, cache, params)
    T = DT[dtype]
    U = torch.empty(max(n * W, 1), dtype=T, device=dev)
    D = torch.empty_like(U)
    rec = dict(exit=torch.empty(sc.dim, max(n * W, 1), dtype=T, device=dev),
               w1=torch.empty(max(n * W, 1), dtype=T, device=dev),
               steps=torch.empty(max(n * W, 1), dtype=torch.int32, device=dev) if records else None)
    counters = torch.zeros(4, dtype=torch.int64, device=dev)
    if started is not None:
        started.record()
    B.bvc_cache_walks(sc.h, params, n, cache.x, cache.nrm, cache.R0, cache.xbar, U, D, rec["exit"], rec["w1"],
                      rec["steps"], counters)
    return U, D, rec, counters


def _set_cache_order(sc: Scene, cache: Cache, params: B.bvc_walk_params):
    """The cache walks start in the cache points' spatial order (once per
    cache; up to the device count when there is one)."""
    if cache.cap and cache.order is None and sc.ordered_walks:
        cache.order = sc.spatial_order(cache.x, cache.cap, cache.n_dev)
    if cache.order is not None:
        params.order = cache.order.data_ptr()


def pointwise(sc: Scene, params: B.bvc_walk_params, x, with_grad=True, order=None):
    """Pointwise walk on spheres at points x ([dim][n] of the walk dtype):
    returns (u [n], grad [dim][n] or None, counters).  order: the points'
    launch order (Scene.spatial_order), or None."""
    dev, d = sc.device, sc.dim
    n = x.shape[1] if x.dim() == 2 else 0
    if order is not None and n:
        params.order = order.data_ptr()
    W = params.n_walks
    T = x.dtype
    Uw = torch.empty(max(n * W, 1), dtype=T, device=dev)
    Gw = torch.empty(d, max(n * W, 1), dtype=T, device=dev) if with_grad else None
    nbytes = B.bvc_pointwise_workspace_bytes(d, max(n, 1), W, B.dtype_code(T), with_grad)
    work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    u = torch.empty(max(n, 1), dtype=T, device=dev)
    g = torch.empty(d, max(n, 1), dtype=T, device=dev) if with_grad else None
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    B.bvc_pointwise_wos(sc.h, params, n, x, Uw, Gw, work, u, g, cnt)
    return u, g, cnt


def reduce_walks(cache: Cache, W, U, D, dtype_out="f32"):
    dev = U.device
    n = cache.cap
    uhat = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    dudn = torch.empty_like(uhat)
    a = torch.empty(max(n, 1), dtype=DT[dtype_out], device=dev)
    b = torch.empty_like(a)
    if cache.n_dev is None:
        B.bvc_reduce_walks(n, W, B.dtype_code(U.dtype), U, D, cache.w, uhat, dudn, CODE[dtype_out], a, b)
    else:
        B.bvc_reduce_walks_count(n, cache.n_dev, W, B.dtype_code(U.dtype), U, D, cache.w, uhat, dudn,
                                 CODE[dtype_out], a, b)
    return uhat, dudn, a, b


def sample_sources(sc: Scene, f: DeviceField, m, l, seed, batch=0, lo=None, hi=None):
    d, dev = sc.dim, sc.device
    M = m**d
    y = torch.empty(d, max(M, 1), dtype=torch.float64, device=dev)
    s = torch.empty(max(M, 1), dtype=torch.float64, device=dev)
    B.bvc_sample_sources(sc.h, f.c(), m, lo if lo is not None else sc.lo, hi if hi is not None else sc.hi, l,
                         seed, batch, y, s)
    return y, s, M


def classify(sc: Scene, x64, l):
    n = x64.shape[1]
    cls = torch.empty(max(n, 1), dtype=torch.int32, device=sc.device)
    dist = torch.empty(max(n, 1), dtype=torch.float64, device=sc.device)
    B.bvc_classify(sc.h, n, x64, l, cls, dist)
    return cls, dist


@dataclass
class Solution:
    idx_int: torch.Tensor
    n_int: int
    idx_band: torch.Tensor
    n_band: int
    u_int: torch.Tensor
    g_int: Optional[torch.Tensor]
    u_band: torch.Tensor
    g_band: Optional[torch.Tensor]
    cache: Cache
    uhat: torch.Tensor
    dudn: torch.Tensor
    counters: torch.Tensor
    pw_counters: torch.Tensor
    extra: dict = field(default_factory=dict)


class Prepared:
    """Per-scene state reused across solves: device scene, fields, classified
    evaluation points and the candidate count of the cache sampler."""

    def __init__(self, problem, dtype=None, n_cand=None, device="cuda", eval_x=None, clamp=None, near_tau=None,
                 band=None, grad_band=None, grad_band_walks=None, cache_cap=None):
        # points within `band` of the boundary take pointwise walks for u and
        # grad u (the band of Algorithm 1 is the offset l; a wider band trades
        # walks for the gather's error next to the cache surface)
        self.band = float(problem.offset if band is None else band)
        if self.band < problem.offset:
            raise ValueError(f"band {self.band} is narrower than the offset {problem.offset}")
        self.p = problem
        self.dtype = dtype or problem.precision
        self.sc = Scene(problem.scene, device)
        self.g = DeviceField(problem.g, device)
        self.f = DeviceField(problem.f, device) if not problem.f.is_zero else None
        self.n_cand = n_cand or candidates_for(self.sc, problem.n_cache, problem.offset, problem.sides,
                                               problem.seed_cache)
        # a solve keeps its accepted cache count on the device: the arrays
        # have room for n_cap points.  With the candidate count drawn for an
        # expected n_cache accepted points, twice that (plus 1024) lies beyond
        # any plausible draw; a given candidate count may all be accepted.
        if cache_cap is None:
            cache_cap = min(self.n_cand, 2 * problem.n_cache + 1024) if n_cand is None else self.n_cand
        self.n_cap = int(cache_cap)
        self.sc.scratch_int(self.n_cand)
        ex = problem.eval_x if eval_x is None else eval_x
        self.eval64 = torch.from_numpy(np.ascontiguousarray(ex.T)).to(device)
        n = self.eval64.shape[1]
        self.cls, self.dist = classify(self.sc, self.eval64, self.band)
        self.idx_int, self.n_int = self.sc.compact(self.cls, 1)
        self.idx_band, self.n_band = self.sc.compact(self.cls, 2)
        T = DT[self.dtype]
        self.x_int = take(self.eval64, self.idx_int, self.n_int, self.sc.dim, n, T)
        self.x_band = take(self.eval64, self.idx_band, self.n_band, self.sc.dim, n, T)
        self.band_order = (self.sc.spatial_order(self.x_band, self.n_band) if self.n_band and self.sc.ordered_walks
                           else None)
        # which walk launch of a solve starts first when the two overlap (the
        # longer one; tune() measures them): by launch size until then
        self.band_first = self.n_band > self.n_cap
        # FP32 gathers keep the near-singular boundary pairs in FP64: pairs
        # closer than tau (default: the offset l; an evaluation point lies at
        # least l from the boundary and a cache point exactly l from it) are
        # summed from FP64 copies of both points and of the cache values
        self.near_tau = 0.0
        self.x_int64 = None
        self.split = None
        if self.dtype == "f32" and problem.sigma == 0:
            self.near_tau = float(problem.offset if near_tau is None else near_tau)
            if self.near_tau > 0:
                self.x_int64 = take(self.eval64, self.idx_int, self.n_int, self.sc.dim, n, torch.float64)
                self._prepare_split(device)
        self.clamp = None
        if clamp is not None:
            self._prepare_clamp(clamp, device)
        self._prepare_grad_band(grad_band, grad_band_walks, device)

    def _prepare_split(self, device):
        """Only gathered points within l + tau of the boundary can meet a cache
        point closer than tau (every cache point lies l from the boundary).
        The gathered points are reordered once with those first (their count
        is the gather's near_lead, so that the blocks past them skip the near
        test) and the gather's outputs are scattered back to the gathered
        order: the permutation, the permuted coordinates in the gather dtype
        and in FP64."""
        d, n, n_int = self.sc.dim, self.eval64.shape[1], self.n_int
        if n_int == 0:
            return
        cls, _ = classify(self.sc, self.x_int64, self.p.offset + self.near_tau)
        pos_near, n_near = self.sc.compact(cls[:n_int], 2)
        pos_far, n_far = self.sc.compact(cls[:n_int], 1)
        if n_far + n_near != n_int:
            raise RuntimeError("near-field split lost gathered points")
        perm = torch.cat([pos_near[:n_near], pos_far[:n_far]]).contiguous()
        idx = self.idx_int[perm.to(torch.int64)].contiguous()
        self.split = dict(n_near=n_near, perm=perm, x=take(self.eval64, idx, n_int, d, n, DT[self.dtype]),
                          x64=take(self.eval64, idx, n_int, d, n, torch.float64))

    def _prepare_grad_band(self, width, walks, device):
        """Gathered points within `width` of the boundary take grad u from
        pointwise walks (the gradient estimate of Eq. 7 at the point itself)
        in place of the gathered gradient, whose kernels grow like the inverse
        distance to the cache surface squared (2D) or cubed (3D); u stays the
        gathered value.  Found here once: their positions among the gathered
        points and their coordinates in the walk dtype."""
        self.grad_band = 0.0
        self.n_gb = 0
        self.gb_pos = None
        self.x_gb = None
        self.gb_order = None
        self.gb_walks = int(walks or self.p.n_walks)
        if width is None or width <= self.band or self.n_int == 0:
            return
        d, n = self.sc.dim, self.eval64.shape[1]
        self.grad_band = float(width)
        x64 = take(self.eval64, self.idx_int, self.n_int, d, n, torch.float64)
        cls, _ = classify(self.sc, x64, self.grad_band)
        pos, self.n_gb = self.sc.compact(cls[: self.n_int], 2)
        self.gb_pos = pos
        if self.n_gb:
            self.x_gb = take(self.eval64, self.idx_int[pos[: self.n_gb].to(torch.int64)].contiguous(), self.n_gb, d,
                             n, DT[self.dtype])
            self.gb_order = self.sc.spatial_order(self.x_gb, self.n_gb) if self.sc.ordered_walks else None

    def _prepare_clamp(self, clamp, device):
        """Clamped gather with bias correction (Section 3.3, Eq. 8).  clamp:
        dict(c, n_rays, max_hits, seed).  Only gathered points within the
        clamp radius of the offset boundary can receive a correction; they
        are found here once (classification against l + radius) with their
        FP64 coordinates, 2D winding numbers and the correction's workspace."""
        p, sc, d = self.p, self.sc, self.sc.dim
        c = float(clamp["c"])
        r = B.bvc_clamp_radius(d, c)
        n_int = self.n_int
        pos = torch.zeros(1, dtype=torch.int64, device=device)
        n_near = 0
        if n_int:
            x64 = take(self.eval64, self.idx_int, n_int, d, self.eval64.shape[1], torch.float64)
            cls, _ = classify(sc, x64, p.offset + r)
            near, n_near = sc.compact(cls[:n_int], 2)
            pos = near[:max(n_near, 1)].to(torch.int64)
        if n_near:
            xn = take(self.eval64, self.idx_int[pos].contiguous(), n_near, d, self.eval64.shape[1], torch.float64)
        else:
            xn = torch.zeros(d, 1, dtype=torch.float64, device=device)
        wind = None
        if d == 2 and n_near:
            wind = torch.empty(n_near, dtype=torch.int32, device=device)
            B.bvc_point_winding(sc.h, n_near, xn, wind)
        n_rays, max_hits = int(clamp.get("n_rays", 16)), int(clamp.get("max_hits", 4))
        nbytes = B.bvc_clamp_workspace_bytes(d, CODE[self.dtype], n_near, n_rays, max_hits)
        self.clamp = dict(c=c, radius=r, n_near=n_near, pos=pos, x=xn, wind=wind,
                          cp=B.clamp_params(p.offset, p.sides, c, n_rays, max_hits),
                          seed=int(clamp.get("seed", p.seed_walks + 1)),
                          ws=torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device),
                          counters=torch.zeros(6, dtype=torch.int64, device=device))


class RoiPrepared:
    """Region-of-interest caching (Section 3.2, "Boundary Specification"):
    the cache lives on the closed boundary of a region R inside the domain
    (uniform p^dR = 1/|dR|), its walks run on the domain, and only evaluation
    points inside R are gathered (the estimate vanishes outside R).  Sources,
    when the problem has any, are drawn inside R."""

    def __init__(self, problem, roi_scene, dtype=None, n_cand=None, device="cuda", eval_x=None):
        self.p = problem
        self.dtype = dtype or problem.precision
        self.sc = Scene(problem.scene, device)
        self.roi = Scene(roi_scene, device)
        self.g = DeviceField(problem.g, device)
        self.f = DeviceField(problem.f, device) if not problem.f.is_zero else None
        self.n_cand = int(n_cand or problem.n_cache)
        ex = problem.eval_x if eval_x is None else eval_x
        self.eval64 = torch.from_numpy(np.ascontiguousarray(ex.T)).to(device)
        n = self.eval64.shape[1]
        self.cls, self.dist = classify(self.roi, self.eval64, 0.0)
        self.idx_int, self.n_int = self.roi.compact(self.cls, 1)
        self.x_int = take(self.eval64, self.idx_int, self.n_int, self.sc.dim, n, DT[self.dtype])


def solve_roi(prep: RoiPrepared, batch=0, with_grad=True, watch=None) -> Solution:
    """Algorithm 1 on a region of interest: samples on dR, walks on the
    domain, then the gather at the evaluation points inside R."""
    p, sc, roi = prep.p, prep.sc, prep.roi
    dt, d = prep.dtype, sc.dim
    T = DT[dt]
    watch = watch or _NoWatch()
    with watch.stage("sample_cache"):
        cache = sample_roi(sc, roi, prep.n_cand, p.seed_cache, batch)
    wp = walk_params(p.eps, p.n_walks, p.seed_walks, prep.g, prep.f, dt, batch, sigma=p.sigma, side_read=p.side_read)
    with watch.stage("cache_walks"):
        U, D, rec, counters = cache_walks(sc, cache, wp, dt)
    with watch.stage("reduce_walks"):
        uhat, dudn, a, b = reduce_walks(cache, p.n_walks, U, D, dt)
    n = cache.cap
    if T != torch.float64:
        cx = take(cache.x, None, n, d, n, T, count=cache.n_dev)
        cn = take(cache.nrm, None, n, d, n, T, count=cache.n_dev)
    else:
        cx, cn = cache.x, cache.nrm
    cview = dict(n=n, dtype=CODE[dt], x=cx, nrm=cn, a=a, b=b, n_dev=cache.n_dev)
    sview = None
    if prep.f is not None and p.n_sources > 0:
        m = int(round(p.n_sources ** (1.0 / d)))
        with watch.stage("sample_sources"):
            y64, s64, M = sample_sources(roi, prep.f, m, 0.0, p.seed_sources, batch)
            y = take(y64, None, M, d, M, T) if T != torch.float64 else y64
            s = take(s64, None, M, 1, M, T) if T != torch.float64 else s64
        sview = dict(n=M, dtype=CODE[dt], y=y, s=s)
    n_int = prep.n_int
    u_int = torch.empty(max(n_int, 1), dtype=T, device=sc.device)
    g_int = torch.empty(d, max(n_int, 1), dtype=T, device=sc.device) if with_grad else None
    with watch.stage("gather"):
        if with_grad:
            B.bvc_gather_grad(d, cview, sview, n_int, prep.x_int, u_int, g_int, sigma=p.sigma)
        else:
            B.bvc_gather_u(d, cview, sview, n_int, prep.x_int, u_int, sigma=p.sigma)
    empty = torch.zeros(1, dtype=T, device=sc.device)
    return Solution(prep.idx_int, n_int, torch.zeros(1, dtype=torch.int32, device=sc.device), 0, u_int, g_int,
                    empty, None, cache, uhat, dudn, counters, torch.zeros(4, dtype=torch.int64, device=sc.device),
                    extra=dict(U=U, D=D, a=a, b=b, cview=cview, sview=sview, rec=rec))


class MixedPrepared:
    """Boundary value caching with a Neumann part (Section 3.2, "Boundary
    Specification"; 2D, Neumann data h = 0, no source): cache points on the
    offset Dirichlet boundary (walks on stars from a first ball, u and
    du/dn by Eq. 7) and on the Neumann part beyond distance l (walks on stars
    from the boundary, u; du/dn = h = 0); evaluation points farther than l
    from the Dirichlet part are gathered from the cache, the others take
    pointwise walks on stars.  `problem.extra` holds the Dirichlet and the
    Neumann segment sets ("dirichlet", "neumann") of `problem.scene`."""

    def __init__(self, problem, dtype=None, n_cand=None, device="cuda", eval_x=None, n_walks_band=None):
        self.p = problem
        self.dtype = dtype or problem.precision
        self.full = Scene(problem.scene, device)
        self.dir = Scene(problem.extra["dirichlet"], device)
        self.neu = Scene(problem.extra["neumann"], device)
        self.g = DeviceField(problem.g, device)
        self.n_cand = int(n_cand or problem.n_cache)
        self.W_band = int(n_walks_band or problem.n_walks)
        ex = problem.eval_x if eval_x is None else eval_x
        self.eval64 = torch.from_numpy(np.ascontiguousarray(ex.T)).to(device)
        n = self.eval64.shape[1]
        self.cls = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.dist = torch.empty(max(n, 1), dtype=torch.float64, device=device)
        B.bvc_classify_mixed(self.full.h, self.dir.h, n, self.eval64, problem.offset, self.cls, self.dist)
        self.idx_int, self.n_int = self.full.compact(self.cls[:n] if n else self.cls, 1)
        self.idx_band, self.n_band = self.full.compact(self.cls[:n] if n else self.cls, 2)
        T = DT[self.dtype]
        self.x_int = take(self.eval64, self.idx_int, self.n_int, 2, n, T)
        self.x_band = take(self.eval64, self.idx_band, self.n_band, 2, n)
        self.ones_band = torch.ones(max(self.n_band, 1), dtype=torch.float64, device=device)
        self.ws = torch.empty(max(B.bvc_wost_workspace_bytes(self.neu.h), 256), dtype=torch.uint8, device=device)
        # the band walks run beside the cache walks: a workspace of their own
        self.ws_band = torch.empty_like(self.ws)


def sample_mixed(prep: MixedPrepared, seed, batch=0):
    """Mixed cache samples, compacted with the offset points first: returns
    (cache, n_offset)."""
    dev, n_cand = prep.full.device, prep.n_cand
    f64 = torch.float64
    x = torch.empty(2, n_cand, dtype=f64, device=dev)
    nrm = torch.empty_like(x)
    xbar = torch.empty_like(x)
    w = torch.empty(n_cand, dtype=f64, device=dev)
    R0 = torch.empty_like(w)
    kind = torch.empty(n_cand, dtype=torch.int32, device=dev)
    B.bvc_sample_mixed(prep.full.h, prep.dir.h, prep.neu.h, n_cand, prep.p.offset, seed, batch, x, nrm, w, xbar, R0,
                       kind, junction_drop=prep.p.junction_drop)
    idx = torch.empty(n_cand + 1, dtype=torch.int32, device=dev)
    scratch = prep.full.scratch_int(n_cand)
    n0 = B.bvc_compact(n_cand, kind, 1, idx, scratch)
    n1 = B.bvc_compact(n_cand, kind, 2, idx[n0:], scratch)
    n = n0 + n1
    c = Cache(n, take(x, idx, n, 2, n_cand), take(nrm, idx, n, 2, n_cand), take(w, idx, n, 1, n_cand),
              take(xbar, idx, n, 2, n_cand), take(R0, idx, n, 1, n_cand), n_cand)
    return c, n0


def _part(t, lo, hi):
    """Columns [lo, hi) of a [rows][n] tensor as a contiguous [rows][hi - lo]."""
    if t.dim() == 1:
        return t[lo:hi] if hi > lo else t[:1]
    return t[:, lo:hi].contiguous() if hi > lo else t[:, :1].contiguous()


def wost(prep: MixedPrepared, params: B.bvc_walk_params, mode, n, x, nrm=None, R0=None, xbar=None, dtype="f32",
         stream=None, ws=None):
    W = params.n_walks
    T = DT[dtype]
    dev = prep.full.device
    U = torch.empty(max(n * W, 1), dtype=T, device=dev)
    D = torch.empty_like(U)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    B.bvc_wost_walks(prep.dir.h, prep.neu.h, params, mode, n, x, nrm, R0, xbar, U, D, None,
                     prep.ws if ws is None else ws, cnt, stream)
    return U, D, cnt


NEUMANN_BATCH_BIT = 0x80000000  # batch word of the walks from Neumann cache points
GRAD_BAND_BATCH_BIT = 0x40000000  # batch word of the pointwise gradient walks near the boundary


def solve_mixed(prep: MixedPrepared, batch=0, with_grad=True, watch=None) -> Solution:
    """Algorithm 1 with a Neumann part: samples, walks on stars from both
    parts of the cache, per-point means, the gather at the points farther
    than l from the Dirichlet part, pointwise walks on stars within l."""
    p = prep.p
    dt = prep.dtype
    T = DT[dt]
    dev = prep.full.device
    watch = watch or _NoWatch()
    W = p.n_walks
    with watch.stage("sample_cache"):
        cache, n0 = sample_mixed(prep, p.seed_cache, batch)
    n, n1 = cache.n, cache.n - n0
    wp0 = walk_params(p.eps, W, p.seed_walks, prep.g, None, dt, batch, side_read=p.side_read)
    wp1 = walk_params(p.eps, W, p.seed_walks, prep.g, None, dt, batch | NEUMANN_BATCH_BIT, side_read=p.side_read)
    nb = prep.n_band
    main = torch.cuda.current_stream()
    started = torch.cuda.Event() if nb else None
    with watch.stage("cache_walks"):
        if started is not None:
            started.record()
        U0, D0, c0 = wost(prep, wp0, 0, n0, _part(cache.x, 0, n0), _part(cache.nrm, 0, n0), _part(cache.R0, 0, n0),
                          _part(cache.xbar, 0, n0), dt)
        U1, D1, c1 = wost(prep, wp1, 3, n1, _part(cache.x, n0, n), _part(cache.nrm, n0, n), None, None, dt)
    Ub = None
    side = None
    if not nb:
        u_band = torch.empty(1, dtype=T, device=dev)
        pw = torch.zeros(4, dtype=torch.int64, device=dev)
    else:
        # the band walks need nothing from the cache: they run on a second
        # stream (default priority) once the longer cache walks are queued,
        # and fill the CUs those leave
        side = prep.__dict__.setdefault("_band_stream", torch.cuda.Stream())
        side.wait_event(started)
        wpb = walk_params(p.eps, prep.W_band, p.seed_walks, prep.g, None, dt, batch, side_read=p.side_read)
        with torch.cuda.stream(side):
            with watch.stage("band_walks"):
                Ub, Db, pw = wost(prep, wpb, 1, nb, prep.x_band, dtype=dt, ws=prep.ws_band)
                u_band = torch.empty(nb, dtype=T, device=dev)
                ub64 = torch.empty(nb, dtype=torch.float64, device=dev)
                db64 = torch.empty_like(ub64)
                bb = torch.empty(nb, dtype=T, device=dev)
                B.bvc_reduce_walks(nb, prep.W_band, B.dtype_code(T), Ub, Db, prep.ones_band, ub64, db64, CODE[dt],
                                   u_band, bb)
    uhat = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    dudn = torch.empty_like(uhat)
    a = torch.empty(max(n, 1), dtype=T, device=dev)
    b = torch.empty_like(a)
    with watch.stage("reduce_walks"):
        B.bvc_reduce_walks(n0, W, B.dtype_code(T), U0, D0, cache.w, uhat, dudn, CODE[dt], a, b)
        if n1:
            B.bvc_reduce_walks(n1, W, B.dtype_code(T), U1, D1, cache.w[n0:], uhat[n0:], dudn[n0:], CODE[dt], a[n0:],
                               b[n0:])
    if T != torch.float64:
        cx = take(cache.x, None, n, 2, n, T)
        cn = take(cache.nrm, None, n, 2, n, T)
    else:
        cx, cn = cache.x, cache.nrm
    cview = dict(n=n, dtype=CODE[dt], x=cx, nrm=cn, a=a, b=b)
    n_int = prep.n_int
    u_int = torch.empty(max(n_int, 1), dtype=T, device=dev)
    g_int = torch.empty(2, max(n_int, 1), dtype=T, device=dev) if with_grad else None
    with watch.stage("gather"):
        if with_grad:
            B.bvc_gather_grad(2, cview, None, n_int, prep.x_int, u_int, g_int)
        else:
            B.bvc_gather_u(2, cview, None, n_int, prep.x_int, u_int)
    if side is not None:
        main.wait_stream(side)
    return Solution(prep.idx_int, n_int, prep.idx_band, nb, u_int, g_int, u_band, None, cache, uhat, dudn,
                    c0 + c1, pw, extra=dict(n_offset=n0, U0=U0, D0=D0, U1=U1, Ub=Ub, a=a, b=b, cview=cview))


class SceneBatch:
    """Many scenes sharing one launch sequence (bvc_batch_plan / _launch).

    Each entry is (problem, n_eval_candidates) with a Laplace or Poisson
    problem in FP32; caches are drawn once here, evaluation points classified,
    and bvc_batch_launch then runs walks, boundary data, means and the gather
    of every scene with five kernels, which a caller may capture in a graph.
    """

    def __init__(self, problems, device="cuda", cache_batch=0):
        self.entries = []
        items = []
        for p in problems:
            sc = Scene(p.scene, device)
            g = DeviceField(p.g, device)
            f = DeviceField(p.f, device) if not p.f.is_zero else None
            n_cand = candidates_for(sc, p.n_cache, p.offset, p.sides, p.seed_cache)
            cache = sample_cache(sc, n_cand, p.offset, p.sides, p.seed_cache, cache_batch)
            d = sc.dim
            cx = take(cache.x, None, cache.n, d, max(cache.n, 1), torch.float32)
            cn = take(cache.nrm, None, cache.n, d, max(cache.n, 1), torch.float32)
            ex64 = torch.from_numpy(np.ascontiguousarray(p.eval_x.T)).to(device)
            cls, _ = classify(sc, ex64, p.offset)
            idx, n_int = sc.compact(cls, 1)
            x_int = take(ex64, idx, n_int, d, ex64.shape[1], torch.float32)
            u = torch.empty(max(n_int, 1), dtype=torch.float32, device=device)
            wp = walk_params(p.eps, p.n_walks, p.seed_walks, g, f, "f32", cache_batch)
            it = B.bvc_batch_item()
            it.scene = sc.h
            it.walk = wp
            it.n_cache = cache.n
            it.x, it.nrm, it.R0, it.xbar, it.w = (t.data_ptr() for t in (cache.x, cache.nrm, cache.R0, cache.xbar,
                                                                          cache.w))
            it.cx, it.cn = cx.data_ptr(), cn.data_ptr()
            it.n_eval = n_int
            it.eval_x = x_int.data_ptr()
            it.u = u.data_ptr()
            items.append(it)
            self.entries.append(dict(problem=p, scene=sc, g=g, f=f, cache=cache, cx=cx, cn=cn, x=x_int, n_int=n_int,
                                     idx=idx, u=u, params=wp))
        self.items = items
        nbytes = B.bvc_batch_workspace_bytes(items)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.h = B.bvc_batch_plan(items, self.ws)

    def __del__(self):
        try:
            B.bvc_batch_destroy(self.h)
        except Exception:
            pass

    def launch(self):
        B.bvc_batch_launch(self.h)

    def counters(self):
        """The batch's uint64[4] counters (work queue, queries, capped, walks)."""
        off = B.bvc_batch_counters(self.h) - self.ws.data_ptr()
        return self.ws[off:off + 32].view(torch.int64).cpu().numpy()

    def results(self):
        """Per scene (U, D, a, b) after a launch: FP32 per-walk samples
        [n_cache*W] and cache values [n_cache], views of the workspace."""
        ptrs = B.bvc_batch_results(self.h)
        base = self.ws.data_ptr()
        total_w = sum(e["cache"].n * e["problem"].n_walks for e in self.entries)
        total_c = sum(e["cache"].n for e in self.entries)
        views = []
        for p, n in zip(ptrs, (total_w, total_w, total_c, total_c)):
            off = p - base
            assert off >= 0 and off % 4 == 0 and off + 4 * n <= self.ws.numel()
            views.append(self.ws[off:off + 4 * n].view(torch.float32))
        out, wo, co = [], 0, 0
        for e in self.entries:
            nw, nc = e["cache"].n * e["problem"].n_walks, e["cache"].n
            out.append((views[0][wo:wo + nw], views[1][wo:wo + nw], views[2][co:co + nc], views[3][co:co + nc]))
            wo += nw
            co += nc
        return out

    def run_sequential(self):
        """The same work with one call sequence per scene (walks, means, gather)."""
        outs = []
        for e in self.entries:
            p, sc, cache = e["problem"], e["scene"], e["cache"]
            U, D, rec, _ = cache_walks(sc, cache, e["params"], "f32")
            uhat, dudn, a, b = reduce_walks(cache, p.n_walks, U, D, "f32")
            u = torch.empty(max(e["n_int"], 1), dtype=torch.float32, device=sc.device)
            cview = dict(n=cache.n, dtype=B.F32, x=e["cx"], nrm=e["cn"], a=a, b=b)
            B.bvc_gather_u(sc.dim, cview, None, e["n_int"], e["x"], u)
            outs.append(u)
        return outs


class Stopwatch:
    """HIP events around named stages on torch's current stream (the stream
    every library call is enqueued on)."""

    def __init__(self):
        self.marks = []

    def stage(self, name):
        sw = self

        class _Ctx:
            def __enter__(self):
                self.e0 = torch.cuda.Event(enable_timing=True)
                self.e1 = torch.cuda.Event(enable_timing=True)
                self.e0.record()
                return self

            def __exit__(self, *exc):
                self.e1.record()
                sw.marks.append((name, self.e0, self.e1))
                return False

        return _Ctx()

    def kernel(self, name, params: B.bvc_walk_params):
        """Times the walk kernel of the call that takes `params` alone: the
        library records the two events right around its launch."""
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()  # creates the events; the library records them again
        e1.record()
        params.ev_begin = e0.cuda_event
        params.ev_end = e1.cuda_event
        self.marks.append((name, e0, e1))

    def totals_ms(self):
        out = {}
        for name, e0, e1 in self.marks:
            out.setdefault(name, []).append(e0.elapsed_time(e1))
        return out


class _NoWatch:
    class _N:
        def __enter__(self):
            return self

        def __exit__(self, *exc):
            return False

    def stage(self, name):
        return self._N()

    def kernel(self, name, params):
        pass


def _gather_views(prep: Prepared, cache: Cache, a, b, batch, watch):
    """Cache view (positions and normals in the gather dtype, a, b) and the
    source view (jittered source samples, Eq. 4) of one solve."""
    p, sc, dt = prep.p, prep.sc, prep.dtype
    T, d = DT[dt], sc.dim
    n = cache.cap
    if T != torch.float64:
        cx = take(cache.x, None, n, d, n, T, count=cache.n_dev)
        cn = take(cache.nrm, None, n, d, n, T, count=cache.n_dev)
    else:
        cx, cn = cache.x, cache.nrm
    cview = dict(n=n, dtype=CODE[dt], x=cx, nrm=cn, a=a, b=b, n_dev=cache.n_dev)
    sview = None
    if prep.f is not None and p.n_sources > 0:
        m = int(round(p.n_sources ** (1.0 / d)))
        with watch.stage("sample_sources"):
            y64, s64, M = sample_sources(sc, prep.f, m, p.offset, p.seed_sources, batch)
            if T != torch.float64:
                y = take(y64, None, M, d, M, T)
                s = take(s64, None, M, 1, M, T)
            else:
                y, s = y64, s64
        sview = dict(n=M, dtype=CODE[dt], y=y, s=s)
    return cview, sview


def _near(prep: Prepared, cache: Cache, U, D):
    """Near-field argument of an FP32 gather (None when off): FP64 cache
    values a, b from the walks' FP64 means, and the FP64 cache points,
    normals and evaluation points (reordered, with the near-field points
    leading, when the gathered points were reordered)."""
    if not prep.near_tau or cache.cap == 0:
        return None
    _, _, a64, b64 = reduce_walks(cache, prep.p.n_walks, U, D, "f64")
    sp = prep.split
    if sp is not None:
        return dict(tau=prep.near_tau, x=sp["x64"], cx=cache.x, cn=cache.nrm, a=a64, b=b64, lead=sp["n_near"])
    return dict(tau=prep.near_tau, x=prep.x_int64, cx=cache.x, cn=cache.nrm, a=a64, b=b64)


def gather_all(prep: Prepared, cview, sview, u_int, g_int, near, clamp=0.0, sigma=0.0):
    """The gather at every gathered point; with the near-field split, over the
    reordered points (those that can need the near field first) and scattered
    back into u_int (and g_int)."""
    d = prep.sc.dim
    sp = prep.split
    if sp is None or near is None:
        x, u, g = prep.x_int, u_int, g_int
    else:
        x = sp["x"]
        u = torch.empty_like(u_int)
        g = torch.empty_like(g_int) if g_int is not None else None
    if g is not None:
        B.bvc_gather_grad(d, cview, sview, prep.n_int, x, u, g, clamp=clamp, sigma=sigma, near=near)
    else:
        B.bvc_gather_u(d, cview, sview, prep.n_int, x, u, clamp=clamp, sigma=sigma, near=near)
    if u is not u_int:
        code = B.dtype_code(u.dtype)
        B.bvc_scatter(code, prep.n_int, sp["perm"], 1, u.shape[0], u, u_int.shape[0], u_int)
        if g is not None:
            B.bvc_scatter(code, prep.n_int, sp["perm"], d, g.shape[1], g, g_int.shape[1], g_int)

def tune(prep: Prepared, with_grad=True, reps=3) -> dict:
    """Picks the launch shapes of this problem's walks and gather with the
    library's tuners (bvc_tune_walks, bvc_tune_gather) on one solve's real
    inputs; later solves of the same problem class use them.  Results do not
    depend on the shapes."""
    p, sc, dt = prep.p, prep.sc, prep.dtype
    T, d = DT[dt], sc.dim
    cache = sample_cache_device(sc, prep.n_cand, prep.n_cap, p.offset, p.sides, p.seed_cache, 0)
    wp = walk_params(p.eps, p.n_walks, p.seed_walks, prep.g, prep.f, dt, 0, sigma=p.sigma,
                     open_sphere=p.extra.get("open_sphere"), side_read=p.side_read)
    wp.n_dev = cache.n_dev.data_ptr()
    _set_cache_order(sc, cache, wp)
    n, W = cache.cap, p.n_walks
    U = torch.empty(max(n * W, 1), dtype=T, device=sc.device)
    D = torch.empty_like(U)
    ex = torch.empty(d, max(n * W, 1), dtype=T, device=sc.device)
    w1 = torch.empty_like(U)
    counters = torch.zeros(4, dtype=torch.int64, device=sc.device)
    bpc, lanes, slabs = B.bvc_tune_walks(sc.h, wp, n, cache.x, cache.nrm, cache.R0, cache.xbar, U, D, ex, w1, counters,
                                  reps)
    cache_ms = _launch_ms(wp, lambda: B.bvc_cache_walks(sc.h, wp, n, cache.x, cache.nrm, cache.R0, cache.xbar, U, D,
                                                        ex, w1, None, counters))
    _, _, a, b = reduce_walks(cache, W, U, D, dt)
    cview, sview = _gather_views(prep, cache, a, b, 0, _NoWatch())
    u = torch.empty(max(prep.n_int, 1), dtype=T, device=sc.device)
    g = torch.empty(d, max(prep.n_int, 1), dtype=T, device=sc.device) if with_grad else None
    near = _near(prep, cache, U, D)
    x = prep.split["x"] if prep.split is not None and near is not None else prep.x_int
    ppt = (B.bvc_tune_gather(d, cview, sview, prep.n_int, x, u, g, reps, near=near)
           if prep.n_int and p.sigma == 0 else 0)
    out = dict(walk_blocks_per_cu=bpc, walk_open_lanes=lanes, walk_slabs=slabs, gather_points_per_thread=ppt)
    nb = prep.n_band
    if nb:
        # the band points' pointwise walks: another class with its own shape
        wpb = walk_params(p.eps, p.n_walks, p.seed_walks, prep.g, prep.f, dt, 0, sigma=p.sigma,
                          open_sphere=p.extra.get("open_sphere"), side_read=p.side_read)
        xb = prep.x_band[:, :nb].contiguous()
        Uw = torch.empty(nb * p.n_walks, dtype=T, device=sc.device)
        Gw = torch.empty(d, nb * p.n_walks, dtype=T, device=sc.device) if with_grad else None
        work = torch.empty(B.bvc_pointwise_workspace_bytes(d, nb, p.n_walks, B.dtype_code(T), with_grad),
                           dtype=torch.uint8, device=sc.device)
        ub = torch.empty(nb, dtype=T, device=sc.device)
        gb = torch.empty(d, nb, dtype=T, device=sc.device) if with_grad else None
        cnt = torch.zeros(4, dtype=torch.int64, device=sc.device)
        if prep.band_order is not None:
            wpb.order = prep.band_order.data_ptr()
        bpb, lb, sb = B.bvc_tune_pointwise(sc.h, wpb, nb, xb, Uw, Gw, work, ub, gb, cnt, reps)
        band_ms = _launch_ms(wpb, lambda: B.bvc_pointwise_wos(sc.h, wpb, nb, xb, Uw, Gw, work, ub, gb, cnt))
        prep.band_first = band_ms > cache_ms
        out.update(band_blocks_per_cu=bpb, band_open_lanes=lb, band_slabs=sb, band_first=prep.band_first)
    return out


def _launch_ms(params: B.bvc_walk_params, launch) -> float:
    """Duration of one walk launch in ms (events the library records right
    around its kernel)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    e1.record()
    params.ev_begin, params.ev_end = e0.cuda_event, e1.cuda_event
    launch()
    params.ev_begin = params.ev_end = None
    e1.synchronize()
    return e0.elapsed_time(e1)


def solve(prep: Prepared, batch=0, with_grad=True, n_walks_band=None, records=False, watch=None) -> Solution:
    p, sc = prep.p, prep.sc
    dt = prep.dtype
    T = DT[dt]
    d = sc.dim
    watch = watch or _NoWatch()
    osph = p.extra.get("open_sphere")
    Wb = n_walks_band or p.n_walks
    nb = prep.n_band
    wpb = walk_params(p.eps, Wb, p.seed_walks, prep.g, prep.f, dt, batch, sigma=p.sigma, open_sphere=osph,
                      side_read=p.side_read)
    band = None
    main = torch.cuda.current_stream()
    # the band walks need nothing from the cache: once it is sampled they run
    # on a second stream (default priority) beside the cache walks and the
    # gather.  The longer of the two walk launches starts first and holds the
    # GPU at its own speed; the shorter fills the CUs its blocks leave.
    side = prep.__dict__.setdefault("_band_stream", torch.cuda.Stream()) if nb else None

    def launch_band():
        watch.kernel("k_walks_band", wpb)
        with torch.cuda.stream(side):
            return pointwise(sc, wpb, prep.x_band[:, :nb], with_grad, order=prep.band_order)

    with watch.stage("sample_cache"):
        cache = sample_cache_device(sc, prep.n_cand, prep.n_cap, p.offset, p.sides, p.seed_cache, batch)
    if side is not None and prep.band_first:
        side.wait_stream(main)
        band = launch_band()
    wp = walk_params(p.eps, p.n_walks, p.seed_walks, prep.g, prep.f, dt, batch, sigma=p.sigma, open_sphere=osph,
                     side_read=p.side_read)
    watch.kernel("k_walks_cache", wp)
    started = torch.cuda.Event() if side is not None and band is None else None
    with watch.stage("cache_walks"):
        U, D, rec, counters = cache_walks(sc, cache, wp, dt, records, started=started)
    if started is not None:
        side.wait_event(started)
        band = launch_band()
    with watch.stage("reduce_walks"):
        uhat, dudn, a, b = reduce_walks(cache, p.n_walks, U, D, dt)
        near = _near(prep, cache, U, D)
    cview, sview = _gather_views(prep, cache, a, b, batch, watch)
    n_int = prep.n_int
    u_int = torch.empty(max(n_int, 1), dtype=T, device=sc.device)
    g_int = torch.empty(d, max(n_int, 1), dtype=T, device=sc.device) if with_grad else None
    cl = prep.clamp
    cc = cl["c"] if cl else 0.0
    with watch.stage("gather"):
        gather_all(prep, cview, sview, u_int, g_int, near, clamp=cc, sigma=p.sigma)
    gathered = None
    if cl:
        gathered = torch.cuda.Event()
        gathered.record()
    if band is None:
        watch.kernel("k_walks_band", wpb)
        with watch.stage("band_walks"):
            u_band, g_band, pwc = pointwise(sc, wpb, prep.x_band[:, :nb] if nb else prep.x_band[:, :0], with_grad,
                                            order=prep.band_order)
    else:
        main.wait_stream(side)
        u_band, g_band, pwc = band
    gb = None
    if with_grad and prep.n_gb:
        # pointwise gradients near the boundary replace the gathered ones
        wpg = walk_params(p.eps, prep.gb_walks, p.seed_walks, prep.g, prep.f, dt, batch | GRAD_BAND_BATCH_BIT,
                          sigma=p.sigma, open_sphere=osph, side_read=p.side_read)
        watch.kernel("k_walks_grad_band", wpg)
        with watch.stage("grad_band_walks"):
            _, gg, gbc = pointwise(sc, wpg, prep.x_gb, True, order=prep.gb_order)
            B.bvc_scatter(B.dtype_code(T), prep.n_gb, prep.gb_pos, d, gg.shape[1], gg, g_int.shape[1], g_int)
        gb = dict(n=prep.n_gb, width=prep.grad_band, walks=prep.gb_walks, counters=gbc)
    if cl:
        # the second integral of Eq. 8 at the gathered points near the offset
        # boundary, on a third stream (default priority) as soon as the gather
        # is done, beside what remains of the band walks; it reads the
        # gather's output
        main = torch.cuda.current_stream()
        side = cl.setdefault("stream", torch.cuda.Stream())
        side.wait_event(gathered)
        wpc = walk_params(p.eps, 1, cl["seed"], prep.g, prep.f, dt, batch, side_read=p.side_read)
        with torch.cuda.stream(side):
            with watch.stage("clamp_correction"):
                B.bvc_clamp_correction(sc.h, wpc, cl["cp"], cl["n_near"], cl["x"], cl["wind"], cl["pos"], u_int,
                                       cl["ws"], cl["counters"])
        main.wait_stream(side)
    return Solution(prep.idx_int, n_int, prep.idx_band, nb, u_int, g_int, u_band, g_band, cache, uhat, dudn,
                    counters, pwc, extra=dict(U=U, D=D, a=a, b=b, cview=cview, sview=sview, rec=rec, near=near,
                                              grad_band=gb))
