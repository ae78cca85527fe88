"""Benchmark: Boundary Value Caching on one MI355X.

The headline line is the 3D Laplace workload: a displaced icosphere of 81,920
triangles with solid-harmonic boundary data (degree <= 8).  One step is one
pass of the whole hot path: 65,536 cache points on the offset boundary, 512
walks each, FP64 cache means, the gather of u at every interior point of a
1,048,576-point uniform sample plus a 256^2 slice, and pointwise walks for the
points within l of the boundary.  The 2D Poisson workload (4096-segment
self-intersecting star, 16,384 cache points x 256 walks, u and grad u on a
1024^2 grid, 128^2 Gaussian sources) runs after it and is reported under the
key "c2" with the same fields.  Inputs are synthetic and seeded (no dataset
exists for this method); each scene is built and uploaded once before timing.

Each workload reports: interior points per second of the BVC step, walk
steps per second, the error of the BVC result against the closed form next to
pointwise walk on spheres at matching error, the memory roofline of the
longest kernel (the walks, on algorithmic traversal bytes) with its VALU
bound, the VALU roofline of the gather, and the FP64 oracle timed on the host
cores (all threads and one thread).
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
# lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_LANE_OPS = 256 * 64 * 2.4e9

# Algorithmic FP operations per gather pair (transcendentals count 1): 2D u
# and grad u, boundary entry (Eqs. 3 and 5) and source entry (Eqs. 4 and 6);
# 3D u, boundary entry (Eq. 3): difference (3), r^2 (5), rsqrt (1), r^-2 and
# r^-3 (2), n.(y - x) (5), the two terms and their accumulation (4).
FLOPS_2D_BOUNDARY_UG = 26
FLOPS_2D_SOURCE_UG = 14
FLOPS_3D_BOUNDARY_U = 20

# Minimal VALU lane-operations of one walk step (one closest-point query and
# the sphere jump that follows it), counted from the arithmetic of each part:
# a Philox-4x32-10 block is ten rounds of two 32-bit multiplies in high and
# low halves, four xors and two key additions; a node expansion is two child
# boxes (per axis: two differences, a three-way max against 0 and a
# multiply-add) plus the ordering of the two; a segment is the clamped
# projection and its squared distance; a triangle is the face-region closest
# point (edge vectors, six dot products, barycentric weights, the point and
# its squared distance); the step itself draws the direction, jumps and tests
# the shell.
OPS_PHILOX_BLOCK = 100
OPS_NODE = {2: 22, 3: 30}
OPS_PRIM = {2: 15, 3: 50}
OPS_STEP = {2: 12, 3: 15}
# a 3D node's two slab bounds when the traversal uses them: per child the
# dot product n.p (5), the distance to the range (3) and the comparison with
# the box bound (1), twice
OPS_SLAB = 18


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=1024, help="c2: evaluation grid size")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"], help="c2: walk and gather precision")
    ap.add_argument("--no-pointwise", action="store_true", help="skip the pointwise-WoS comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-c2", action="store_true", help="c3 headline without the c2 line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of each CPU oracle leg")
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c4a", "c4b", "c2clamp", "c3clamp", "c3screen",
                                                    "c2roi", "c2mixed", "c2screen", "c2slit", "c3open"],
                    help="c3 (headline, with c2 under the key 'c2') and c2 print the benchmark line; the others "
                         "print their own measurement lines")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (no autotuning)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-captured replay of the step")
    ap.add_argument("--clamp-c", type=float, default=20.0, help="c2clamp: bound c of dG/dn (Eq. 9)")
    ap.add_argument("--clamp-rays", type=int, default=64, help="c2clamp: rays per corrected point")
    ap.add_argument("--clamp-hits", type=int, default=4, help="c2clamp: contributing crossings kept per ray")
    ap.add_argument("--grad-band", default="1.5,4",
                    help="c2: also solve once per width with pointwise grad u within that many offsets l of the "
                         "boundary (comma-separated; empty: skip)")
    ap.add_argument("--wide-band", default="1.25,2",
                    help="also solve once per width with pointwise walks (u, grad u) within that many offsets l "
                         "(comma-separated; empty: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB device-to-device before timing (HBM counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2))) if len(a) else float("nan")


# bins of the distance to the boundary, in units of the offset l
BIN_EDGES = (0.0, 1.0, 1.25, 1.5, 2.0, 3.0, 4.0, 8.0, math.inf)


def error_by_distance(l, dist, u, truth, g=None, gtrue=None, pointwise=None):
    """RMSE of u (and of grad u, as the root of the mean squared vector
    error) against the closed form in bins of d / l, d the distance to the
    boundary; `pointwise` marks the points whose value (u in [0, 1), grad u
    wherever set) came from pointwise walks."""
    out = []
    r = dist / l
    for lo, hi in zip(BIN_EDGES[:-1], BIN_EDGES[1:]):
        m = (r >= lo) & (r < hi)
        row = {"d_over_l": [lo, hi if math.isfinite(hi) else None], "points": int(m.sum()),
               "rmse_u": rmse(u[m], truth[m])}
        if g is not None:
            row["rmse_grad"] = float(np.sqrt(np.mean(np.sum((g[m] - gtrue[m]) ** 2, 1)))) if m.any() else float("nan")
        if pointwise is not None:
            row["pointwise_points"] = int(pointwise[m].sum())
        out.append(row)
    return out


def band_options(args, pl, prob, prep, dtype, with_grad, base):
    """Cost and effect of two wider bands next to the timed configuration,
    each solved once more (same cache, sources, streams and points): grad u
    from pointwise walks within args.grad_band l (u still gathered), and
    pointwise u and grad u within args.wide_band l.  `base` holds the sampled
    points' truth of the timed run (indices into the evaluation points)."""
    import torch

    l = prob.offset
    out = {}
    opts = []
    if with_grad:
        opts += [(f"grad_band_{w:g}l", "grad_band", dict(grad_band=w * l)) for w in widths(args.grad_band)]
    opts += [(f"wide_band_{w:g}l", "wide_band", dict(band=w * l)) for w in widths(args.wide_band)]
    for name, key, kw in opts:
        p2 = pl.Prepared(prob, dtype=dtype, n_cand=prep.n_cand, **kw)
        pl.solve(p2, batch=args.steps - 1, with_grad=with_grad)
        torch.cuda.synchronize()
        watch = pl.Stopwatch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s2 = pl.solve(p2, batch=args.steps - 1, with_grad=with_grad, watch=watch)
        e1.record()
        torch.cuda.synchronize()
        u, g, pw = gather_values(p2, s2, with_grad)
        idx = base["idx"]
        row = {"width_over_l": kw.get("grad_band", kw.get("band")) / l, "step_ms": round(e0.elapsed_time(e1), 4),
               "stage_ms": {k: round(float(np.mean(v)), 4) for k, v in watch.totals_ms().items()
                            if not k.startswith("k_")},
               "pointwise_points": int(p2.n_gb if key == "grad_band" else p2.n_band),
               "walks_per_point": int(p2.gb_walks if key == "grad_band" else prob.n_walks),
               "by_distance": error_by_distance(l, base["dist"], u[idx], base["truth"],
                                                g[idx] if g is not None else None, base.get("gtrue"), pw[idx])}
        row["rmse_u_all"] = rmse(u[idx], base["truth"])
        if g is not None:
            row["rmse_grad_all"] = float(np.sqrt(np.mean(np.sum((g[idx] - base["gtrue"]) ** 2, 1))))
        out[name] = row
        log(f"{name}: {row['pointwise_points']} points, step {row['step_ms']} ms")
        del p2, s2
    return out


def widths(spec):
    return [float(w) for w in str(spec).split(",") if w.strip() and float(w) > 1]


def gather_values(prep, sol, with_grad):
    """u (and grad u) of one solve at every evaluation point (NaN outside),
    and a mask of the points whose grad u came from pointwise walks."""
    n = prep.eval64.shape[1]
    d = prep.sc.dim
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy().astype(np.int64)
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy().astype(np.int64)
    u = np.full(n, np.nan)
    u[idx_i] = sol.u_int[: prep.n_int].double().cpu().numpy()
    u[idx_b] = sol.u_band[: prep.n_band].double().cpu().numpy()
    g = None
    pw = np.zeros(n, bool)
    pw[idx_b] = True
    if with_grad:
        g = np.full((n, d), np.nan)
        g[idx_i] = sol.g_int[:, : prep.n_int].double().cpu().numpy().T
        g[idx_b] = sol.g_band[:, : prep.n_band].double().cpu().numpy().T
        if getattr(prep, "n_gb", 0):
            pw[idx_i[prep.gb_pos[: prep.n_gb].cpu().numpy().astype(np.int64)]] = True
    return u, g, pw


def measured_traffic(kernel, workload, sources):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel's sources have
    changed since those counters were taken (their SHA-256 is recorded beside
    the figure)."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel: " + re.escape(kernel) + r"\s+workload: " + re.escape(workload) +
                  r"\s+source_sha256: ([0-9a-f]{64})\s+traffic_bytes_per_launch: (\d+)", text)
    if not m:
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2302_11825_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m.group(2)) if h.hexdigest() == m.group(1) else None


GATHER_SOURCES = ("kernels_gather.hip", "bvc_device.hpp", "bvc_internal.hpp")
WALK_SOURCES = ("walks.hip", "bvc_device.hpp", "bvc_internal.hpp", "scene.cpp")  # the tree the walks read


def walk_bytes(dim, es, mode, with_grad, slabs=True):
    """Algorithmic bytes of the walk kernel in the record sizes of FP32 (es =
    4; FP64 doubles them): per binary BVH node expanded, 48 B in 2D and 64 B
    in 3D (two child boxes and their links), plus in 3D, when the traversal
    uses them, the 40 B of the two children's slab bounds (axis and range
    each); per primitive tested, a 16 B segment or a 36 B triangle; per walk,
    its inputs read and records written (mode 0 cache walk, mode 1 pointwise
    walk)."""
    s = es // 4
    node = (48 if dim == 2 else 64 + (40 if slabs else 0)) * s
    prim = (16 if dim == 2 else 36) * s
    if mode == 0:
        io = 8 + 2 * dim * 8 + dim * es + 3 * es          # R0, x, n (FP64); exit, U, D, w1
    else:
        io = 8 + dim * es + dim * es + es + (2 * dim * es if with_grad else 0)  # R0, x; exit, U, grad, w1
    return node, prim, io


def philox_blocks_per_step(dim, src):
    """Philox blocks a walk step evaluates: the direction, plus the in-ball
    source point of a Poisson walk (two blocks in 2D, three in 3D)."""
    return 1 + ((2 if dim == 2 else 3) if src else 0)


def walk_roofline(kernel, dim, es, mode, with_grad, ms, queries, walks, work_key, work, src, traffic, slabs=True):
    """Memory roofline of one walk launch on algorithmic traversal bytes (the
    nodes and primitives a nearest-first query visits, counted by the oracle
    on this BVH, times their record sizes, plus each walk's inputs and
    records), and its VALU bound: the minimal lane-operations of those
    visits, the Philox blocks and the step arithmetic, against the chip's
    lane-operation peak."""
    slabs = bool(slabs) and dim == 3
    node_b, prim_b, io_b = walk_bytes(dim, es, mode, with_grad, slabs)
    ops_node = OPS_NODE[dim] + (OPS_SLAB if slabs else 0)
    out = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
           "traffic": traffic, "kernel": kernel, "avg_launch_ms": round(ms, 4), "queries_per_launch": queries,
           "walks_per_launch": walks, "bytes": {"node": node_b, "primitive": prim_b, "walk_io": io_b}}
    valu = None
    if work is not None and ms > 0:
        vn, vp = work[work_key]["nodes_per_query"], work[work_key]["prims_per_query"]
        per_query = vn * node_b + vp * prim_b
        alg = queries * per_query + walks * io_b
        gbs = alg / (ms / 1e3) / 1e9
        out.update(achieved=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4), nodes_per_query=vn,
                   prims_per_query=vp, bytes_per_query=round(per_query, 1), bytes_per_launch=alg)
        if gbs > PEAK_HBM_GBS:
            out["note"] = ("the algorithmic bytes outrun the HBM peak: L2 and the MALL serve the traversal data "
                           "(traffic counts only what missed L2), so HBM does not bind; the kernel's limit is "
                           "VALU issue (roofline_valu)")
        ops = (philox_blocks_per_step(dim, src) * OPS_PHILOX_BLOCK + OPS_STEP[dim] + vn * ops_node +
               vp * OPS_PRIM[dim])
        rate = queries * ops / (ms / 1e3)
        valu = {"bound": "valu", "achieved": rate / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                "frac": round(rate / PEAK_LANE_OPS, 4), "kernel": kernel, "lane_ops_per_query": round(ops, 1),
                "ops": {"philox_block": OPS_PHILOX_BLOCK, "philox_blocks_per_step": philox_blocks_per_step(dim, src),
                        "node": ops_node, "primitive": OPS_PRIM[dim], "step": OPS_STEP[dim]}}
        out["slab_bounds"] = slabs
    return out, valu


def near_field_effect(pl, prep, sol, with_grad, truth_i, sel, dist_i, gather_ms):
    """Cost and effect of the FP64 near field of the timed FP32 gather: the
    same gather launched once more without it (same cache, sources and
    points), its time and the error of both near the boundary."""
    import torch

    from paper_2302_11825_amd import _bvc as B

    near = sol.extra.get("near")
    if near is None or prep.n_int == 0:
        return None
    d = prep.sc.dim
    cview, sview = sol.extra["cview"], sol.extra["sview"]
    u0 = torch.empty_like(sol.u_int)
    g0 = torch.empty_like(sol.g_int) if with_grad else None
    fn = ((lambda: B.bvc_gather_grad(d, cview, sview, prep.n_int, prep.x_int, u0, g0)) if with_grad else
          (lambda: B.bvc_gather_u(d, cview, sview, prep.n_int, prep.x_int, u0)))
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    ms_off = e0.elapsed_time(e1)
    u_on = sol.u_int[: prep.n_int].double().cpu().numpy()[sel]
    u_off = u0[: prep.n_int].double().cpu().numpy()[sel]
    close = dist_i < 2 * near["tau"] + prep.p.offset
    return {"tau": near["tau"], "gather_ms_with": round(gather_ms, 4), "gather_ms_without": round(ms_off, 4),
            "points_within_l_plus_2tau": int(close.sum()),
            "rmse_there_with": rmse(u_on[close], truth_i[close]), "rmse_there_without": rmse(u_off[close], truth_i[close]),
            "max_abs_change": float(np.abs(u_on - u_off).max()) if u_on.size else 0.0}


def pointwise_curve(pl, prob, prep, dtype, pts, truth, rmse_bvc, value):
    """Pointwise walk on spheres on a subset of interior points at 1 to 256
    walks per point; the walks per point that match BVC's error come from the
    fit rmse^2 = a/W + b^2, and the time per walk from the largest run."""
    import torch

    xs = torch.from_numpy(np.ascontiguousarray(pts.T)).to("cuda", pl.DT[dtype])
    ks = xs.shape[1]
    curve = []
    for Wp in (1, 4, 16, 64, 256):
        wp = pl.walk_params(prob.eps, Wp, prob.seed_walks + 1, prep.g, prep.f, dtype)
        pl.pointwise(prep.sc, wp, xs, with_grad=False)  # warm
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        uo, _, cnt = pl.pointwise(prep.sc, wp, xs, with_grad=False)
        a1.record()
        torch.cuda.synchronize()
        ms = a0.elapsed_time(a1)
        curve.append({"walks": Wp, "rmse": rmse(uo.double().cpu().numpy()[:ks], truth), "ms": ms,
                      "points_per_s": ks / (ms / 1e3), "steps": int(cnt[1])})
    Ws = np.array([c["walks"] for c in curve], float)
    r2 = np.array([c["rmse"] for c in curve]) ** 2
    # least squares relative to each point's own size, so that every W counts
    A = np.stack([1 / Ws, np.ones_like(Ws)], 1) / r2[:, None]
    (a_fit, b2_fit), *_ = np.linalg.lstsq(A, np.ones_like(r2), rcond=None)
    b2_fit = max(b2_fit, 0.0)
    target = rmse_bvc**2
    w_star = a_fit / (target - b2_fit) if target > b2_fit and a_fit > 0 else float("inf")
    per_walk_ms = curve[-1]["ms"] / curve[-1]["walks"]
    pw_pts_s = ks / (max(w_star, 1.0) * per_walk_ms / 1e3) if math.isfinite(w_star) else 0.0
    return {"subset": ks, "rmse_bvc_subset": rmse_bvc, "curve": curve,
            "fit": {"a": float(a_fit), "b2": float(b2_fit)},
            "walks_for_equal_rmse": (float(w_star) if math.isfinite(w_star) else None),
            "points_per_s_at_equal_rmse": pw_pts_s,
            "bvc_over_pointwise": (value / pw_pts_s if pw_pts_s > 0 else None)}


def timed_steps(pl, prep, args, with_grad):
    """Warm-up steps, then exactly args.steps steps between two events, with
    the host garbage collector off and each step's buffers released before
    the next, so that the caching allocator reuses them."""
    import torch

    for w in range(args.warmup):
        pl.solve(prep, batch=1000 + w, with_grad=with_grad)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    counts = []
    cache_counts = []
    sol = None
    gc.collect()
    gc.disable()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for s in range(args.steps):
        sol = None
        sol = pl.solve(prep, batch=s, with_grad=with_grad, watch=watch)
        counts.append((sol.counters, sol.pw_counters))
        cache_counts.append(sol.cache.n_dev)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    ms_step = e0.elapsed_time(e1) / args.steps
    timers = {k: float(np.mean(v)) for k, v in watch.totals_ms().items()}
    # every step's accepted cache count fitted its capacity
    worst = max(int(c[0]) for c in cache_counts) if cache_counts else 0
    if worst > prep.n_cap:
        raise RuntimeError(f"cache overflow in a timed step: {worst} > {prep.n_cap}")
    return sol, counts, ms_step, wall, timers


def captured_step(pl, prep, args, with_grad):
    """The step captured once in a HIP graph (it has no host synchronisation:
    the cache count stays on the device) and replayed args.steps times
    between two events.  The graph holds the kernel arguments of one batch,
    so every replay redoes that batch's work."""
    import torch

    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pl.solve(prep, batch=0, with_grad=with_grad)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        sol = pl.solve(prep, batch=0, with_grad=with_grad)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    out = {"ms_per_step": round(ms, 4), "replays": args.steps, "cache_points": sol.cache.n}
    del graph, sol
    torch.cuda.empty_cache()
    return out


def run_workload(args, which):
    """One benchmark line (without the process-level keys) for c2 or c3."""
    import torch

    import workloads as wl
    from paper_2302_11825_amd import pipeline as pl

    dim = 3 if which == "c3" else 2
    dtype = "f32" if which == "c3" else args.dtype
    with_grad = which == "c2"
    t_setup = time.time()
    prob = wl.problem_c3() if which == "c3" else wl.problem_c2(grid=args.grid)
    prep = pl.Prepared(prob, dtype=dtype)
    tuned = None if args.no_tune else pl.tune(prep, with_grad=with_grad, reps=1 if dim == 3 else 3)
    torch.cuda.synchronize()
    setup_s = time.time() - t_setup
    log(f"{which} setup {setup_s:.1f}s: candidates {prep.n_cand}, interior {prep.n_int}, band {prep.n_band}")
    if args.calib_copy_mib > 0:
        # a plain copy of known size: the reference that scales HBM counters
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sol, counts, ms_step, wall, timers = timed_steps(pl, prep, args, with_grad)
    captured = None if args.no_graph else captured_step(pl, prep, args, with_grad)
    if captured:
        log(f"{which} captured step {captured['ms_per_step']} ms (eager {ms_step:.3f} ms)")
    kernels = {k: v for k, v in timers.items() if k.startswith("k_")}
    stages = {k: v for k, v in timers.items() if not k.startswith("k_")}
    log(f"{which} timed {args.steps} steps: {ms_step:.2f} ms/step (wall {wall:.2f}s) {stages}")

    n_pts = prep.n_int + prep.n_band
    value = n_pts / (ms_step / 1e3)
    steps_total = sum(int(c[1]) + int(p[1]) for c, p in counts)
    walks_total = sum(int(c[3]) + int(p[3]) for c, p in counts)
    capped = sum(int(c[2]) + int(p[2]) for c, p in counts)
    cache_ms = kernels.get("k_walks_cache", stages.get("cache_walks", 0.0))
    band_ms = kernels.get("k_walks_band", stages.get("band_walks", 0.0))
    cache_steps = sum(int(c[1]) for c, _ in counts) / args.steps

    # error of the last step against the closed form (3D: an even sample of
    # about 200k points, the solid harmonics being costly to evaluate)
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    stride = max(1, idx_i.size // 200000) if dim == 3 else 1
    sel = np.arange(0, idx_i.size, stride)
    pts_i = prob.eval_x[idx_i[sel]]
    pts_b = prob.eval_x[idx_b]
    truth_i = wl.field_value(prob.truth, pts_i)
    truth_b = wl.field_value(prob.truth, pts_b)
    u_i = sol.u_int[: prep.n_int].double().cpu().numpy()[sel]
    u_b = sol.u_band[: prep.n_band].double().cpu().numpy()
    dist_i = prep.dist[idx_i[sel]].cpu().numpy() if prep.n_int else np.zeros(0)
    far = dist_i >= 0.05
    err = {"all": rmse(np.concatenate([u_i, u_b]), np.concatenate([truth_i, truth_b])),
           "gathered": rmse(u_i, truth_i), "gathered_d_ge_0.05": rmse(u_i[far], truth_i[far]),
           "band": rmse(u_b, truth_b), "rms_true": float(np.sqrt(np.mean(truth_i**2)))}
    if dim == 3:
        err["sample"] = f"every {stride}th gathered point ({sel.size}) and every band point"
    # by distance to the boundary: the sampled gathered points and every band
    # point (2D: grad u against finite differences of the closed form)
    base = {"idx": np.concatenate([idx_i[sel], idx_b]).astype(np.int64),
            "dist": np.concatenate([dist_i, prep.dist[idx_b].cpu().numpy() if prep.n_band else np.zeros(0)]),
            "truth": np.concatenate([truth_i, truth_b])}
    u_all, g_all, pw_all = gather_values(prep, sol, with_grad)
    if with_grad:
        base["gtrue"] = wl.field_grad_fd(prob.truth, prob.eval_x[base["idx"]], 1e-6)
        gerr = np.sum((g_all[base["idx"]] - base["gtrue"]) ** 2, axis=1)
        gi = gerr[: sel.size]
        err["grad"] = float(np.sqrt(np.mean(gi)))
        err["grad_d_ge_0.05"] = float(np.sqrt(np.mean(gi[far]))) if far.any() else float("nan")
        err["grad_band"] = float(np.sqrt(np.mean(gerr[sel.size:]))) if prep.n_band else float("nan")
    err["by_distance"] = error_by_distance(prob.offset, base["dist"], u_all[base["idx"]], base["truth"],
                                           g_all[base["idx"]] if with_grad else None, base.get("gtrue"),
                                           pw_all[base["idx"]])
    err["by_distance_note"] = ("d_over_l: bin of the distance to the boundary in offsets l; [0, 1) are the band "
                               "points (pointwise walks), the rest gathered")
    if widths(args.grad_band) or widths(args.wide_band):
        err["band_options"] = band_options(args, pl, prob, prep, dtype, with_grad, base)

    # VALU roofline of the gather (one launch per step)
    gather_ms = stages["gather"]
    n_src = int(sol.extra["sview"]["n"]) if sol.extra["sview"] else 0
    pairs_b = prep.n_int * sol.cache.n
    pairs_s = prep.n_int * n_src
    if dim == 2:
        flops = pairs_b * FLOPS_2D_BOUNDARY_UG + pairs_s * FLOPS_2D_SOURCE_UG
        fpp = {"boundary": FLOPS_2D_BOUNDARY_UG, "source": FLOPS_2D_SOURCE_UG}
    else:
        flops = pairs_b * FLOPS_3D_BOUNDARY_U
        fpp = {"boundary": FLOPS_3D_BOUNDARY_U}
    achieved = flops / (gather_ms / 1e3) / 1e12
    # the gather's template names its evaluation points per thread: the tuned
    # value, else the library's default of 2
    ppt = tuned["gather_points_per_thread"] if tuned else 2
    T = "float" if dtype == "f32" else "double"
    near_on = "true" if sol.extra.get("near") is not None else "false"
    gather_kernel = f"k_gather<{T},{dim},{'true' if with_grad else 'false'},{near_on},{ppt},false>"
    roofline_gather = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                       "traffic": measured_traffic(gather_kernel, which, GATHER_SOURCES),
                       "kernel": gather_kernel, "pairs_per_launch": pairs_b + pairs_s, "flops_per_pair": fpp,
                       "avg_launch_ms": round(gather_ms, 4), "pairs_per_s": (pairs_b + pairs_s) / (gather_ms / 1e3)}

    near_field = near_field_effect(pl, prep, sol, with_grad, truth_i, sel, dist_i, gather_ms)

    pointwise = None
    if not args.no_pointwise and prep.n_int > 0:
        rng = np.random.default_rng(wl.seed(2 if dim == 2 else 3, 5))
        sub = np.sort(rng.choice(sel.size, size=min(8192, sel.size), replace=False))
        pointwise = pointwise_curve(pl, prob, prep, dtype, pts_i[sub], truth_i[sub], rmse(u_i[sub], truth_i[sub]),
                                    value)
        log(f"{which} pointwise {pointwise['walks_for_equal_rmse']} walks for equal RMSE")

    # the traversal's slab bounds (3D): the tuned choices (default of a
    # bounded domain: on)
    cache_slabs = bool((tuned or {}).get("walk_slabs", 1)) and dim == 3
    band_slabs = bool((tuned or {}).get("band_slabs", 1)) and dim == 3
    cpu, work = None, None
    if not args.no_cpu:
        cpu, work = oracle_leg(prob, prep, sol, args.cpu_seconds, n_pts, dim, with_grad, pointwise,
                               (cache_slabs, band_slabs))
        log(f"{which} cpu baseline {cpu}")

    es = 4 if dtype == "f32" else 8
    src = prob.f.kind != 0
    T = "float" if es == 4 else "double"
    if dim == 3:
        # the cache walks are the longest launch of the 3D step
        kname = f"k_walks<{T},3,false,0>"
        roofline, valu = walk_roofline(kname + " (cache walks)", 3, es, 0, False, cache_ms, int(sol.counters[1]),
                                       int(sol.counters[3]), "cache", work, src,
                                       measured_traffic(kname, which, WALK_SOURCES) if es == 4 else None,
                                       cache_slabs)
        other, other_valu = walk_roofline(f"k_walks<{T},3,false,1> (band-point walks)", 3, es, 1, False, band_ms,
                                          int(sol.pw_counters[1]), int(sol.pw_counters[3]), "band", work, src, None,
                                          band_slabs)
    else:
        # the band-point walks are the longest launch of the 2D step
        kname = f"k_walks<{T},2,true,1>"
        roofline, valu = walk_roofline(kname + " (band-point walks)", 2, es, 1, True, band_ms,
                                       int(sol.pw_counters[1]), int(sol.pw_counters[3]), "band", work, src,
                                       measured_traffic(kname, which, WALK_SOURCES) if es == 4 else None)
        other, other_valu = walk_roofline(f"k_walks<{T},2,true,0> (cache walks)", 2, es, 0, False, cache_ms,
                                          int(sol.counters[1]), int(sol.counters[3]), "cache", work, src, None)
    if work is not None:
        roofline["counted_on"] = work["counted_on"]
    if prep.n_band:
        # the two walk launches of a step overlap on two streams
        first = prep.band_first == (dim == 2)
        roofline["overlap"] = ("the other walk launch runs beside this one on a second stream; this one "
                               + ("starts first" if first else "starts second and its duration includes the wait"))

    config = {"workload": prob.name, "primitives": int(prob.scene.prims.shape[0]),
              "cache_target": prob.n_cache, "cache_candidates": prep.n_cand, "cache_points": sol.cache.n,
              "cache_capacity": prep.n_cap,
              "walks_per_point": prob.n_walks, "interior_points": prep.n_int, "band_points": prep.n_band,
              "eps": prob.eps, "offset_l": prob.offset}
    if dim == 2:
        config.update(grid=f"{args.grid}x{args.grid}", sources=n_src)
    else:
        config.update(evaluation=f"{prob.extra['n_box']} uniform box candidates + {prob.extra['n_slice']}-point "
                                 f"z = 0 slice, classified")
    return {
        "metric": "interior pts/sec at fixed RMSE (BVC vs pointwise WoS); walk steps/sec",
        "value": value,
        "unit": "points/s",
        "ms_per_step": ms_step,
        "dtype": dtype,
        "config": config,
        "walk_steps_per_s": steps_total / (ms_step * args.steps / 1e3),
        "cache_walk_steps_per_s": cache_steps / (cache_ms / 1e3) if cache_ms > 0 else 0.0,
        "walks_per_step": walks_total / args.steps,
        "capped_walks": capped,
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        "kernel_ms": {k: round(v, 4) for k, v in kernels.items()},
        "rmse": err,
        "pointwise_wos": pointwise,
        "roofline": roofline,
        "roofline_valu": valu,
        "roofline_other_walks": {"hbm": other, "valu": other_valu},
        "roofline_gather": roofline_gather,
        "near_field": near_field,
        "captured_step": captured,
        "cpu_baseline": cpu,
        "setup_s": setup_s,
        "tuned_shapes": tuned,
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2302_11825_amd import pipeline as pl  # noqa: F401  (fails loudly without libbvc.so)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload not in ("c2", "c3"):
        from paper_2302_11825_amd import measure

        measure.run(args)
        return
    line = run_workload(args, args.workload)
    out = {"metric": line.pop("metric"), "value": line.pop("value"), "unit": line.pop("unit"), "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": line.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": line.pop("dtype"),
           "data": "synthetic", "config": line.pop("config")}
    out.update(line)
    if args.workload == "c3" and not args.no_c2:
        gc.collect()
        torch.cuda.empty_cache()
        out["c2"] = run_workload(args, "c2")
    print(json.dumps(out))


_NATIVE = None


def native_oracle():
    """The oracle built on this host with -O3 -march=native (same arithmetic:
    no FMA contraction, no reassociation), loaded for the timing legs."""
    global _NATIVE
    import oracle

    if _NATIVE is None:
        path = os.path.join(tempfile.mkdtemp(prefix="bvc_oracle_"), "liboracle_native.so")
        oracle.build(path=path, native=True)
        oracle.load(path)
        _NATIVE = path
    return oracle


def oracle_leg(prob, prep, sol, budget_s, n_pts, dim, with_grad, pointwise, slabs=(True, True)):
    """The host oracle leg.  (1) cpu_baseline: the FP64 oracle, built here
    with -O3 -march=native -ffp-contract=off, on a bounded sample of the same
    step, extrapolated to the step's full work: walks of the first cache
    points, the gather at the first interior points against the whole cache
    and source set, pointwise walks at the first band points; once on all
    host threads and once on one thread.  BVC against pointwise walk on
    spheres on the oracle: the oracle's pointwise walks at interior points,
    times the walks per point that match BVC's error (the estimator's
    property, measured on the GPU).  (2) The traversal work per
    closest-point query: the oracle replays walks with the library's walk ids
    and counts the nodes and primitives a nearest-first query visits on the
    library's own BVH (exported through the C-ABI)."""
    oracle = native_oracle()
    osc = oracle.Scene(prob.scene)
    W = prob.n_walks
    n_cache = sol.cache.n
    cn = {k: np.ascontiguousarray(v.cpu().numpy()[:, :n_cache].T) if v.dim() == 2 else v.cpu().numpy()[:n_cache]
          for k, v in dict(x=sol.cache.x, n=sol.cache.nrm, w=sol.cache.w, xbar=sol.cache.xbar,
                           R0=sol.cache.R0).items()}
    sv = sol.extra["sview"]
    sy = np.ascontiguousarray(sv["y"].double().cpu().numpy().T) if sv else None
    sw = sv["s"].double().cpu().numpy() if sv else None
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    P = oracle.walk_params(prob.eps, W, prob.seed_walks)
    all_threads = oracle.num_threads()

    def leg(threads, share):
        oracle.set_threads(threads)
        nw = 1
        while True:
            sub = {k: v[:nw] for k, v in cn.items()}
            t = time.perf_counter()
            out = oracle.cache_walks(osc, prob.g, prob.f, P, sub)
            tw = time.perf_counter() - t
            if tw > share / 4 or nw >= n_cache:
                break
            nw = min(n_cache, nw * 4)
        walks_per_s = nw * W / tw
        uh, dh = oracle.reduce(out["U"], out["D"], W)
        a = np.resize(uh, n_cache) * cn["w"]
        b = np.resize(dh, n_cache) * cn["w"]
        ng = 4
        while True:
            pts = prob.eval_x[idx_i[:ng]]
            t = time.perf_counter()
            oracle.gather(dim, pts, cn["x"], cn["n"], a, b, sy, sw, with_grad=with_grad)
            tg = time.perf_counter() - t
            if tg > share / 4 or ng >= prep.n_int:
                break
            ng = min(prep.n_int, ng * 4)
        gather_pts_s = ng / tg
        nbp = 1
        tb = 0.0
        while prep.n_band:
            t = time.perf_counter()
            oracle.pointwise(osc, prob.g, prob.f, P, prob.eval_x[idx_b[:nbp]], with_grad=with_grad)
            tb = time.perf_counter() - t
            if tb > share / 8 or nbp >= min(prep.n_band, 256):
                break
            nbp = min(prep.n_band, 256, nbp * 4)
        band_pts_s = nbp / tb if tb > 0 else float("inf")
        step_s = (n_cache * W / walks_per_s + prep.n_int / gather_pts_s +
                  (prep.n_band / band_pts_s if prep.n_band else 0.0))
        return {"value": n_pts / step_s, "unit": "points/s", "threads": threads,
                "step_s_extrapolated": step_s, "walks_per_s": walks_per_s, "gather_points_per_s": gather_pts_s,
                "band_points_per_s": band_pts_s,
                "sample": (f"{nw} cache points x {W} walks, gather at {ng} interior points against {n_cache} cache"
                           f" + {0 if sw is None else sw.size} sources, pointwise walks ({W} each) at {nbp} band "
                           f"points; extrapolated to the full step ({step_s:.1f} s)")}

    full = leg(all_threads, budget_s)
    one = leg(1, budget_s / 2)
    oracle.set_threads(all_threads)
    # BVC against pointwise WoS on the oracle
    bvc_vs_pw = None
    if pointwise and pointwise.get("walks_for_equal_rmse"):
        wstar = max(pointwise["walks_for_equal_rmse"], 1.0)
        npw = 1
        while True:
            pts = prob.eval_x[idx_i[: 8 * npw : 8]]
            Pp = oracle.walk_params(prob.eps, 16, prob.seed_walks + 1)
            t = time.perf_counter()
            oracle.pointwise(osc, prob.g, prob.f, Pp, pts, with_grad=False)
            tp = time.perf_counter() - t
            if tp > budget_s / 8 or 8 * npw >= prep.n_int:
                break
            npw *= 4
        pw_walks_s = pts.shape[0] * 16 / tp
        pw_pts_s = pw_walks_s / wstar
        bvc_vs_pw = {"pointwise_walks_per_s": pw_walks_s, "walks_for_equal_rmse": wstar,
                     "pointwise_points_per_s_at_equal_rmse": pw_pts_s, "bvc_points_per_s": full["value"],
                     "bvc_over_pointwise": full["value"] / pw_pts_s,
                     "sample": f"16 pointwise walks at {pts.shape[0]} interior points, all threads"}
    work = traversal_work(oracle, osc, prob, prep, cn, idx_b, W, slabs=slabs)
    cpu = {"value": full["value"], "unit": "points/s", "cores": all_threads, "kind": "oracle",
           "sample": "FP64 oracle, all host threads: " + full["sample"],
           "step_s_extrapolated": full["step_s_extrapolated"], "one_thread": one,
           "all_threads": {k: full[k] for k in ("walks_per_s", "gather_points_per_s", "band_points_per_s")},
           "cpu_model": oracle.cpu_model(), "host_cpus": os.cpu_count(),
           "build": "gcc " + " ".join(oracle.FLAGS + ["-march=native"]),
           "bvc_vs_pointwise_on_oracle": bvc_vs_pw}
    return cpu, work


def traversal_work(oracle, osc, prob, prep, cn, idx_b, W, n_cache_pts=256, n_band_pts=1024, walks_each=8,
                   slabs=(True, True)):
    """Mean nodes expanded and primitives tested per query, counted by the
    oracle on the library's exported BVH (with its slab bounds where the
    cache or band walks use them, `slabs`), over the queries of `walks_each`
    walks (ids i*W + j, as the library numbers them) of cache points and band
    points taken evenly across their sets (cache walks and pointwise walks)."""
    from paper_2302_11825_amd import _bvc as B

    child, boxes, order = B.bvc_scene_export_bvh(prep.sc.h)
    sl = B.bvc_scene_export_slabs(prep.sc.h) if prob.scene.dim == 3 else None
    slabs_cache = sl if slabs[0] else None
    slabs_band = sl if slabs[1] else None
    P = oracle.walk_params(prob.eps, W, prob.seed_walks)
    out = {}
    n_all = cn["x"].shape[0]
    ci = np.linspace(0, n_all - 1, min(n_cache_pts, n_all)).astype(np.int64)
    nc = ci.size
    ids = [int(i) * W + j for i in ci for j in range(walks_each)]
    q, h, _ = oracle.walk_queries(osc, P, 0, np.repeat(cn["x"][ci], walks_each, 0),
                                  np.repeat(cn["R0"][ci], walks_each), ids)
    vn, vp = oracle.bvh_visits(osc, child, boxes, order, q, h, slabs=slabs_cache)
    out["cache"] = {"nodes_per_query": float(vn.mean()), "prims_per_query": float(vp.mean()),
                    "queries_counted": int(q.shape[0])}
    bi = np.linspace(0, idx_b.size - 1, min(n_band_pts, idx_b.size)).astype(np.int64)
    nb = bi.size
    pts = prob.eval_x[idx_b[bi]]
    d, _, _ = osc.closest(pts)
    ids = [int(k) * W + j for k in bi for j in range(walks_each)]
    q, h, _ = oracle.walk_queries(osc, P, 1, np.repeat(pts, walks_each, 0), np.repeat(d, walks_each), ids)
    vn, vp = oracle.bvh_visits(osc, child, boxes, order, q, h, slabs=slabs_band)
    out["band"] = {"nodes_per_query": float(vn.mean()), "prims_per_query": float(vp.mean()),
                   "queries_counted": int(q.shape[0])}
    out["counted_on"] = (f"{out['cache']['queries_counted']} cache-walk and {out['band']['queries_counted']} "
                         f"band-walk queries of oracle walks ({walks_each} walks x {nc} cache / {nb} band points)")
    return out


if __name__ == "__main__":
    main()
