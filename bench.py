"""Benchmark: Boundary Value Caching on one MI355X.

One step is one pass of the whole hot path over the 2D Poisson workload with
a self-intersecting 4096-segment star: cache sampling (16,384 cache points
on the offset boundary), 256 walks per cache point, FP64 cache means, source
samples (128^2 jittered), gather of u and grad u at the interior points of a
1024^2 grid, and pointwise walks for the grid points within l of the
boundary.  Inputs are synthetic and seeded (no dataset exists for this
method); the scene is built and uploaded once before timing.

Prints one JSON line: interior points per second of the BVC step, walk steps
per second, the error of the BVC result against the manufactured closed form
next to pointwise walk on spheres at matching error, the roofline of the
longest kernel of the step (the band-point walks, memory roofline on
algorithmic traversal bytes) and of the gather (VALU roofline), and the FP64
oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0

# Algorithmic FP operations per gather pair (transcendentals count 1), 2D u and
# grad u: boundary entry (Eqs. 3 and 5) and source entry (Eqs. 4 and 6).
FLOPS_2D_BOUNDARY_UG = 26
FLOPS_2D_SOURCE_UG = 14
FLOPS_2D_BOUNDARY_U = 14
FLOPS_2D_SOURCE_U = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-pointwise", action="store_true", help="skip the pointwise-WoS comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4a", "c4b", "c2clamp", "c3clamp", "c3screen", "c2roi",
                                                    "c2mixed", "c2screen", "c2slit", "c3open"],
                    help="c2 prints the benchmark line; the others print their own measurement lines")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (no autotuning)")
    ap.add_argument("--clamp-c", type=float, default=20.0, help="c2clamp: bound c of dG/dn (Eq. 9)")
    ap.add_argument("--clamp-rays", type=int, default=64, help="c2clamp: rays per corrected point")
    ap.add_argument("--clamp-hits", type=int, default=4, help="c2clamp: contributing crossings kept per ray")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB device-to-device before timing (HBM counter calibration)")
    return ap.parse_args()


def rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)))


def measured_traffic(kernel, sources):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel's sources have changed since
    those counters were taken (their SHA-256 is recorded beside the figure)."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "c2_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel: " + re.escape(kernel) + r"\s+source_sha256: ([0-9a-f]{64})\s+"
                  r"traffic_bytes_per_launch: (\d+)", text)
    if not m:
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2302_11825_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m.group(2)) if h.hexdigest() == m.group(1) else None


GATHER_SOURCES = ("kernels_gather.hip", "bvc_device.hpp", "bvc_internal.hpp")
WALK_SOURCES = ("walks.hip", "bvc_device.hpp", "bvc_internal.hpp")


def walk_bytes(dim, es, mode, with_grad):
    """Algorithmic bytes of the walk kernel: per BVH node expanded (two child
    boxes in the walk precision plus the int2 child links), per primitive
    tested (segment: 4 values; triangle: 3 x 4 values), and per walk (inputs
    read and records written; mode 0 cache walk, mode 1 pointwise walk)."""
    node = 2 * 2 * dim * es + 8
    prim = (4 if dim == 2 else 12) * es
    if mode == 0:
        io = 8 + 2 * dim * 8 + dim * es + 3 * es          # R0, x, n (FP64); exit, U, D, w1
    else:
        io = 8 + dim * es + dim * es + es + (2 * dim * es if with_grad else 0)  # R0, x; exit, U, grad, w1
    return node, prim, io


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as wl
    from paper_2302_11825_amd import _bvc as B
    from paper_2302_11825_amd import pipeline as pl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload != "c2":
        from paper_2302_11825_amd import measure

        measure.run(args)
        return
    t_setup = time.time()
    prob = wl.problem_c2(grid=args.grid)
    prep = pl.Prepared(prob, dtype=args.dtype)
    tuned = None if args.no_tune else pl.tune(prep, with_grad=True)
    torch.cuda.synchronize()
    setup_s = time.time() - t_setup
    print(f"[bench] setup {setup_s:.1f}s: candidates {prep.n_cand}, interior {prep.n_int}, band {prep.n_band}",
          file=sys.stderr, flush=True)

    if args.calib_copy_mib > 0:
        # a plain copy of known size: the reference that scales HBM counters
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(args.warmup):
        pl.solve(prep, batch=1000 + w)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    watch = pl.Stopwatch()
    counts = []  # per step: (cache-walk counters, band-walk counters), device tensors
    sol = None
    torch.cuda.synchronize()
    # the host's cyclic garbage collector stays out of the timed region, and
    # each step's buffers are released before the next one so that the
    # caching allocator reuses them instead of growing the pool mid-run
    gc.collect()
    gc.disable()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for s in range(args.steps):
        sol = None
        sol = pl.solve(prep, batch=s, watch=watch)
        counts.append((sol.counters, sol.pw_counters))
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    ms_step = e0.elapsed_time(e1) / args.steps
    timers = {k: float(np.mean(v)) for k, v in watch.totals_ms().items()}
    kernels = {k: v for k, v in timers.items() if k.startswith("k_")}
    stages = {k: v for k, v in timers.items() if not k.startswith("k_")}
    print(f"[bench] timed {args.steps} steps: {ms_step:.2f} ms/step (wall {wall:.2f}s) {stages}",
          file=sys.stderr, flush=True)

    n_pts = prep.n_int + prep.n_band
    value = n_pts / (ms_step / 1e3)
    steps_total = sum(int(c[1]) + int(p[1]) for c, p in counts)
    walks_total = sum(int(c[3]) + int(p[3]) for c, p in counts)
    capped = sum(int(c[2]) + int(p[2]) for c, p in counts)
    walk_ms = kernels.get("k_walks_cache", stages.get("cache_walks", 0.0))
    cache_steps = sum(int(c[1]) for c, _ in counts) / args.steps
    cache_walk_rate = cache_steps / (walk_ms / 1e3) if walk_ms > 0 else 0.0

    # error of the last step against the manufactured closed form
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    pts_i = prob.eval_x[idx_i]
    pts_b = prob.eval_x[idx_b]
    truth_i = wl.field_value(prob.truth, pts_i)
    truth_b = wl.field_value(prob.truth, pts_b)
    u_i = sol.u_int[: prep.n_int].double().cpu().numpy()
    u_b = sol.u_band[: prep.n_band].double().cpu().numpy()
    rmse_all = rmse(np.concatenate([u_i, u_b]), np.concatenate([truth_i, truth_b]))
    rmse_int = rmse(u_i, truth_i)
    dist_i = prep.dist[idx_i].cpu().numpy() if prep.n_int else np.zeros(0)
    far = dist_i >= 0.05
    rmse_far = rmse(u_i[far], truth_i[far]) if far.any() else float("nan")
    grad_true = wl.field_grad_fd(prob.truth, pts_i[::16], 1e-6)
    g_i = sol.g_int[:, : prep.n_int].double().cpu().numpy().T[::16]
    gerr = np.sum((g_i - grad_true) ** 2, axis=1)
    rmse_grad = float(np.sqrt(np.mean(gerr)))
    far16 = far[::16]
    rmse_grad_far = float(np.sqrt(np.mean(gerr[far16]))) if far16.any() else float("nan")
    band_rmse = rmse(u_b, truth_b) if prep.n_band else float("nan")

    # VALU roofline of the gather (one launch per step)
    gather_ms = stages["gather"]
    n_src = int(sol.extra["sview"]["n"]) if sol.extra["sview"] else 0
    pairs_b = prep.n_int * sol.cache.n
    pairs_s = prep.n_int * n_src
    flops = pairs_b * FLOPS_2D_BOUNDARY_UG + pairs_s * FLOPS_2D_SOURCE_UG
    achieved = flops / (gather_ms / 1e3) / 1e12
    # the gather's template names its evaluation points per thread: the tuned
    # value, else the library's default of 2
    ppt = tuned["gather_points_per_thread"] if tuned else 2
    gather_kernel = f"k_gather<float,2,true,false,{ppt},false>"
    roofline_gather = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                       "traffic": measured_traffic(gather_kernel, GATHER_SOURCES),
                       "kernel": gather_kernel, "pairs_per_launch": pairs_b + pairs_s,
                       "flops_per_pair": {"boundary": FLOPS_2D_BOUNDARY_UG, "source": FLOPS_2D_SOURCE_UG},
                       "avg_launch_ms": round(gather_ms, 4),
                       "pairs_per_s": (pairs_b + pairs_s) / (gather_ms / 1e3)}

    # pointwise walk on spheres at matching error, on a subset of interior points
    pointwise = None
    if not args.no_pointwise and prep.n_int > 0:
        rng = np.random.default_rng(wl.seed(2, 5))
        sub = np.sort(rng.choice(prep.n_int, size=min(8192, prep.n_int), replace=False))
        xs = torch.from_numpy(np.ascontiguousarray(pts_i[sub].T)).to("cuda", pl.DT[args.dtype])
        ks = xs.shape[1]
        rmse_bvc_sub = rmse(u_i[sub], truth_i[sub])
        curve = []
        for Wp in (1, 4, 16, 64, 256):
            wp = pl.walk_params(prob.eps, Wp, prob.seed_walks + 1, prep.g, prep.f, args.dtype)
            pl.pointwise(prep.sc, wp, xs, with_grad=False)  # warm
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record()
            uo, _, cnt = pl.pointwise(prep.sc, wp, xs, with_grad=False)
            a1.record()
            torch.cuda.synchronize()
            ms = a0.elapsed_time(a1)
            curve.append({"walks": Wp, "rmse": rmse(uo.double().cpu().numpy(), truth_i[sub]), "ms": ms,
                          "points_per_s": ks / (ms / 1e3), "steps": int(cnt[1])})
        # smallest W with RMSE <= BVC's, from the fit rmse^2 = a/W + b^2
        Ws = np.array([c["walks"] for c in curve], float)
        r2 = np.array([c["rmse"] for c in curve]) ** 2
        # least squares relative to each point's own size, so that every W counts
        A = np.stack([1 / Ws, np.ones_like(Ws)], 1) / r2[:, None]
        (a_fit, b2_fit), *_ = np.linalg.lstsq(A, np.ones_like(r2), rcond=None)
        b2_fit = max(b2_fit, 0.0)
        target = rmse_bvc_sub**2
        w_star = a_fit / (target - b2_fit) if target > b2_fit and a_fit > 0 else float("inf")
        if math.isfinite(w_star):
            # time per walk from the largest run
            per_walk_ms = curve[-1]["ms"] / curve[-1]["walks"]
            pw_pts_s = ks / (max(w_star, 1.0) * per_walk_ms / 1e3)
        else:
            pw_pts_s = 0.0
        pointwise = {"subset": ks, "rmse_bvc_subset": rmse_bvc_sub, "curve": curve,
                     "fit": {"a": float(a_fit), "b2": float(b2_fit)},
                     "walks_for_equal_rmse": (float(w_star) if math.isfinite(w_star) else None),
                     "points_per_s_at_equal_rmse": pw_pts_s,
                     "bvc_over_pointwise": (value / pw_pts_s if pw_pts_s > 0 else None)}
        print(f"[bench] pointwise {pointwise['walks_for_equal_rmse']} walks for equal RMSE", file=sys.stderr,
              flush=True)

    cpu, work = None, None
    if not args.no_cpu:
        cpu, work = oracle_leg(prob, prep, sol, args.cpu_seconds, n_pts)
        print(f"[bench] cpu baseline {cpu}", file=sys.stderr, flush=True)

    # memory roofline of the band-point walk kernel, the longest launch of the
    # step, on algorithmic traversal bytes: nodes and primitives a
    # nearest-first query visits (counted by the oracle on this BVH) times
    # their record sizes, plus each walk's inputs and records
    es = 4 if args.dtype == "f32" else 8
    band_ms = kernels.get("k_walks_band", 0.0)
    q_band, w_band = int(sol.pw_counters[1]), int(sol.pw_counters[3])
    node_b, prim_b, io_b = walk_bytes(2, es, 1, True)
    roofline = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                "traffic": measured_traffic("k_walks<float,2,true,1>", WALK_SOURCES) if es == 4 else None,
                "kernel": "k_walks<float,2,true,1> (band-point walks)", "avg_launch_ms": round(band_ms, 4),
                "queries_per_launch": q_band, "walks_per_launch": w_band,
                "bytes": {"node": node_b, "primitive": prim_b, "walk_io": io_b}}
    walk_rates = {}
    if work is not None and band_ms > 0:
        vn, vp = work["band"]["nodes_per_query"], work["band"]["prims_per_query"]
        per_query = vn * node_b + vp * prim_b
        alg = q_band * per_query + w_band * io_b
        gbs = alg / (band_ms / 1e3) / 1e9
        roofline.update(achieved=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4), nodes_per_query=vn,
                        prims_per_query=vp, bytes_per_query=round(per_query, 1), bytes_per_launch=alg)
        vn_c, vp_c = work["cache"]["nodes_per_query"], work["cache"]["prims_per_query"]
        node_c, prim_c, io_c = walk_bytes(2, es, 0, False)
        q_c, w_c = int(sol.counters[1]), int(sol.counters[3])
        cache_ms = kernels.get("k_walks_cache", 0.0)
        alg_c = q_c * (vn_c * node_c + vp_c * prim_c) + w_c * io_c
        walk_rates = {"cache_walk_kernel": {"avg_launch_ms": round(cache_ms, 4), "queries": q_c,
                                            "nodes_per_query": vn_c, "prims_per_query": vp_c,
                                            "GB_per_s": round(alg_c / (cache_ms / 1e3) / 1e9, 1),
                                            "frac_hbm": round(alg_c / (cache_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)},
                      "counted_on": work["counted_on"]}

    out = {
        "metric": "interior pts/sec at fixed RMSE (BVC vs pointwise WoS); walk steps/sec",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": prob.name, "segments": int(prob.scene.prims.shape[0]),
                   "cache_target": prob.n_cache, "cache_candidates": prep.n_cand,
                   "cache_points": sol.cache.n, "walks_per_point": prob.n_walks, "sources": n_src,
                   "grid": f"{args.grid}x{args.grid}", "interior_points": prep.n_int,
                   "band_points": prep.n_band, "eps": prob.eps, "offset_l": prob.offset},
        "walk_steps_per_s": steps_total / (ms_step * args.steps / 1e3),
        "cache_walk_steps_per_s": cache_walk_rate,
        "walks_per_step": walks_total / args.steps,
        "capped_walks": capped,
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        "rmse": {"all": rmse_all, "gathered": rmse_int, "gathered_d_ge_0.05": rmse_far, "band": band_rmse,
                 "grad": rmse_grad, "grad_d_ge_0.05": rmse_grad_far},
        "pointwise_wos": pointwise,
        "roofline": roofline,
        "roofline_gather": roofline_gather,
        "walk_kernels": walk_rates,
        "kernel_ms": {k: round(v, 4) for k, v in kernels.items()},
        "cpu_baseline": cpu,
        "setup_s": setup_s,
        "tuned_shapes": tuned,
    }
    print(json.dumps(out))


def oracle_leg(prob, prep, sol, budget_s, n_pts):
    """The host oracle leg.  (1) cpu_baseline: the FP64 oracle on a bounded
    sample of the same step, extrapolated to the step's full work: walks of
    the first cache points, the gather at the first interior points,
    pointwise walks at the first band points.  (2) The traversal work per
    closest-point query: the oracle replays walks with the library's walk ids
    and counts the nodes and primitives a nearest-first query visits on the
    library's own BVH (exported through the C-ABI)."""
    import oracle
    import workloads as wl

    osc = oracle.Scene(prob.scene)
    W = prob.n_walks
    n_cache = sol.cache.n
    cn = {k: np.ascontiguousarray(v.cpu().numpy()[:, :n_cache].T) if v.dim() == 2 else v.cpu().numpy()[:n_cache]
          for k, v in dict(x=sol.cache.x, n=sol.cache.nrm, w=sol.cache.w, xbar=sol.cache.xbar,
                           R0=sol.cache.R0).items()}
    share = budget_s / 3
    # walks
    nw = 8
    while True:
        sub = {k: v[:nw] for k, v in cn.items()}
        t = time.perf_counter()
        out = oracle.cache_walks(osc, prob.g, prob.f, oracle.walk_params(prob.eps, W, prob.seed_walks), sub)
        tw = time.perf_counter() - t
        if tw > share / 4 or nw >= n_cache:
            break
        nw = min(n_cache, nw * 4)
    walks_per_s = nw * W / tw
    # gather at interior points against the whole cache and source set
    uh, dh = oracle.reduce(out["U"], out["D"], W)
    a = np.resize(uh, n_cache) * cn["w"]
    b = np.resize(dh, n_cache) * cn["w"]
    sv = sol.extra["sview"]
    sy = np.ascontiguousarray(sv["y"].double().cpu().numpy().T) if sv else None
    sw = sv["s"].double().cpu().numpy() if sv else None
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    ng = 16
    while True:
        pts = prob.eval_x[idx_i[:ng]]
        t = time.perf_counter()
        oracle.gather(2, pts, cn["x"], cn["n"], a, b, sy, sw, with_grad=True)
        tg = time.perf_counter() - t
        if tg > share / 4 or ng >= prep.n_int:
            break
        ng = min(prep.n_int, ng * 4)
    gather_pts_s = ng / tg
    # pointwise walks at band points
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    nbp = min(64, prep.n_band)
    tb = 0.0
    if nbp:
        t = time.perf_counter()
        oracle.pointwise(osc, prob.g, prob.f, oracle.walk_params(prob.eps, W, prob.seed_walks), prob.eval_x[idx_b[:nbp]])
        tb = time.perf_counter() - t
    band_pts_s = nbp / tb if tb > 0 else float("inf")
    step_s = n_cache * W / walks_per_s + prep.n_int / gather_pts_s + (prep.n_band / band_pts_s if nbp else 0.0)
    work = traversal_work(oracle, osc, prob, prep, cn, idx_b, W)
    return {"value": n_pts / step_s, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle: {nw} cache points x {W} walks ({walks_per_s:.3g} walks/s), gather at "
                       f"{ng} interior points against {n_cache} cache + {0 if sw is None else sw.size} sources "
                       f"({gather_pts_s:.3g} points/s), pointwise walks at {nbp} band points; extrapolated to "
                       f"the full step ({step_s:.1f} s)"),
            "step_s_extrapolated": step_s}, work


def traversal_work(oracle, osc, prob, prep, cn, idx_b, W, n_cache_pts=256, n_band_pts=1024, walks_each=8):
    """Mean nodes expanded and primitives tested per query, counted by the
    oracle on the library's exported BVH, over the queries of `walks_each`
    walks (ids i*W + j, as the library numbers them) of cache points and band
    points taken evenly across their sets (cache walks and pointwise walks)."""
    from paper_2302_11825_amd import _bvc as B

    child, boxes, order = B.bvc_scene_export_bvh(prep.sc.h)
    P = oracle.walk_params(prob.eps, W, prob.seed_walks)
    out = {}
    n_all = cn["x"].shape[0]
    ci = np.linspace(0, n_all - 1, min(n_cache_pts, n_all)).astype(np.int64)
    nc = ci.size
    ids = [int(i) * W + j for i in ci for j in range(walks_each)]
    q, h, _ = oracle.walk_queries(osc, P, 0, np.repeat(cn["x"][ci], walks_each, 0),
                                  np.repeat(cn["R0"][ci], walks_each), ids)
    vn, vp = oracle.bvh_visits(osc, child, boxes, order, q, h)
    out["cache"] = {"nodes_per_query": float(vn.mean()), "prims_per_query": float(vp.mean()),
                    "queries_counted": int(q.shape[0])}
    bi = np.linspace(0, idx_b.size - 1, min(n_band_pts, idx_b.size)).astype(np.int64)
    nb = bi.size
    pts = prob.eval_x[idx_b[bi]]
    d, _, _ = osc.closest(pts)
    ids = [int(k) * W + j for k in bi for j in range(walks_each)]
    q, h, _ = oracle.walk_queries(osc, P, 1, np.repeat(pts, walks_each, 0), np.repeat(d, walks_each), ids)
    vn, vp = oracle.bvh_visits(osc, child, boxes, order, q, h)
    out["band"] = {"nodes_per_query": float(vn.mean()), "prims_per_query": float(vp.mean()),
                   "queries_counted": int(q.shape[0])}
    out["counted_on"] = (f"{out['cache']['queries_counted']} cache-walk and {out['band']['queries_counted']} "
                         f"band-walk queries of oracle walks ({walks_each} walks x {nc} cache / {nb} band points)")
    return out


if __name__ == "__main__":
    main()
