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
dominant kernel (the gather), and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
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
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4a", "c4b"],
                    help="c2 prints the benchmark line; the others print their own measurement lines")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB device-to-device before timing (HBM counter calibration)")
    return ap.parse_args()


def rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)))


def measured_traffic():
    """HBM bytes per launch of the gather from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel sources have changed since
    those counters were taken (their SHA-256 is recorded beside the figure)."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "k_gather_c2_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    m_bytes = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m_hash or not m_bytes:
        return None
    h = hashlib.sha256()
    for f in ("kernels_gather.hip", "bvc_device.hpp", "bvc_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2302_11825_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m_bytes.group(1)) if h.hexdigest() == m_hash.group(1) else None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
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
    sols = []
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for s in range(args.steps):
        sols.append(pl.solve(prep, batch=s, watch=watch))
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    stages = {k: float(np.mean(v)) for k, v in watch.totals_ms().items()}
    print(f"[bench] timed {args.steps} steps: {ms_step:.2f} ms/step (wall {wall:.2f}s) {stages}",
          file=sys.stderr, flush=True)

    sol = sols[-1]
    n_pts = prep.n_int + prep.n_band
    value = n_pts / (ms_step / 1e3)
    steps_total = sum(int(s.counters[1]) + int(s.pw_counters[1]) for s in sols)
    walks_total = sum(int(s.counters[3]) + int(s.pw_counters[3]) for s in sols)
    capped = sum(int(s.counters[2]) + int(s.pw_counters[2]) for s in sols)
    walk_ms = stages.get("cache_walks", 0.0)
    cache_steps = sum(int(s.counters[1]) for s in sols) / args.steps
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

    # dominant kernel roofline (the gather: one launch per step)
    gather_ms = stages["gather"]
    n_src = int(sol.extra["sview"]["n"]) if sol.extra["sview"] else 0
    pairs_b = prep.n_int * sol.cache.n
    pairs_s = prep.n_int * n_src
    flops = pairs_b * FLOPS_2D_BOUNDARY_UG + pairs_s * FLOPS_2D_SOURCE_UG
    achieved = flops / (gather_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": measured_traffic(),
                "kernel": "k_gather<float,2,true>", "pairs_per_launch": pairs_b + pairs_s,
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

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(prob, prep, sol, args.cpu_seconds, n_pts)
        print(f"[bench] cpu baseline {cpu}", file=sys.stderr, flush=True)

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
        "cpu_baseline": cpu,
        "setup_s": setup_s,
    }
    print(json.dumps(out))


def cpu_baseline(prob, prep, sol, budget_s, n_pts):
    """The FP64 oracle on a bounded sample of the same step, extrapolated to
    the step's full work: walks of the first cache points, the gather at the
    first interior points, pointwise walks at the first band points."""
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
    return {"value": n_pts / step_s, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle: {nw} cache points x {W} walks ({walks_per_s:.3g} walks/s), gather at "
                       f"{ng} interior points against {n_cache} cache + {0 if sw is None else sw.size} sources "
                       f"({gather_pts_s:.3g} points/s), pointwise walks at {nbp} band points; extrapolated to "
                       f"the full step ({step_s:.1f} s)"),
            "step_s_extrapolated": step_s}


if __name__ == "__main__":
    main()
