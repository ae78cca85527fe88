"""Measurements of the workloads other than the 2D Poisson benchmark line.

    python bench.py --workload c3    3D Laplace, displaced icosphere (81,920 triangles)
    python bench.py --workload c4a   64 boundary-data fields on the 3D walks:
                                     split-BF16 MFMA vs FP32 multi-RHS vs 64 plain gathers
    python bench.py --workload c4b   32 uneven 2D scenes: one graph-replayed launch
                                     sequence vs per-scene call sequences
    python bench.py --workload c2clamp  the 2D Poisson step with the clamped gather
                                     and its bias correction (Section 3.3): time,
                                     and the error near the offset boundary of the
                                     plain, clamped-only and corrected estimates
    python bench.py --workload c3clamp --clamp-c 1600   the same on the 3D Laplace step
    python bench.py --workload c3screen  the 3D step on the screened equation (sigma = 4)
    python bench.py --workload c2screen  the 2D step on the screened equation (sigma = 4)
    python bench.py --workload c3open    the 3D step outside the displaced icosphere, an open
                                     domain (Appendix B), u = 1/|x - q|
    python bench.py --workload c2slit    double-sided Dirichlet data on a cut disk (Appendix B)
    python bench.py --workload c2roi     the 2D Poisson problem cached on the boundary of a
                                     disk inside the star (region of interest, Section 3.2)
    python bench.py --workload c2mixed   Laplace in a channel with Dirichlet ends and Neumann
                                     walls (Section 3.2 with walk on stars), against
                                     pointwise walk on stars at equal error

Each prints one JSON line.  Inputs are the seeded synthetic workloads.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np
import torch

import workloads as wl

from . import _bvc as B
from . import pipeline as pl


# Algorithmic FP operations of one 3D boundary pair for u (Eq. 3): difference
# (3), r^2 (5), rsqrt (1), r^-2 and r^-3 (2), n.(y-x) (5), the two terms and
# their accumulation (4).
FLOPS_3D_BOUNDARY_U = 20


def _ev():
    return torch.cuda.Event(enable_timing=True)


def _time(fn, reps=1):
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _log(msg):
    print(f"[measure] {msg}", file=sys.stderr, flush=True)


def run(args):
    {"c3": c3, "c4a": c4a, "c4b": c4b, "c2clamp": c2clamp, "c3clamp": c3clamp,
     "c3screen": c3screen, "c2roi": c2roi, "c2mixed": c2mixed, "c2screen": c2screen,
     "c2slit": c2slit, "c3open": c3open}[args.workload](args)


def _c3_setup(args, prob=None):
    prob = prob or wl.problem_c3()
    t = time.time()
    prep = pl.Prepared(prob, dtype="f32")
    tuned = None if getattr(args, "no_tune", False) else pl.tune(prep, with_grad=False, reps=1)
    torch.cuda.synchronize()
    _log(f"c3 setup {time.time() - t:.1f}s candidates {prep.n_cand} interior {prep.n_int} band {prep.n_band} "
         f"tuned {tuned}")
    return prob, prep


def c3screen(args):
    """The 3D step on the screened equation Lap u = sigma u (sigma = 4) with the
    plane wave exp(a.x) as data and solution."""
    c3(args, wl.problem_c3_screened())


def c3open(args):
    """The 3D Laplace step in the exterior of the displaced icosphere, an open
    domain (Appendix B): walks escape to infinity (u = 0) or re-enter on a
    sphere enclosing the mesh; data and solution u = 1/|x - q|, q inside the
    solid; evaluation points uniform in [-2, 2]^3."""
    c3(args, wl.problem_c3_open())


def c2slit(args):
    """Double-sided Dirichlet data (Appendix B): the unit disk cut along
    [0, 1] x {0}, u = r^(1/2) cos(phi/2) (sqrt(r) above the cut, -sqrt(r)
    below); 65,536 cache points x 128 walks, 1024^2 grid."""
    prob = wl.problem_slit_disk(grid=args.grid, n_cache=65536, n_walks=128)
    prep = pl.Prepared(prob, dtype="f32")
    torch.cuda.synchronize()
    for _ in range(max(1, args.warmup)):
        pl.solve(prep, with_grad=False)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(args.steps):
        sol = pl.solve(prep, with_grad=False, watch=watch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = {k: sum(v) / len(v) for k, v in watch.totals_ms().items()}
    xi = prob.eval_x[prep.idx_int[: prep.n_int].cpu().numpy()]
    xb = prob.eval_x[prep.idx_band[: prep.n_band].cpu().numpy()]
    ti, tb = wl.field_value(prob.truth, xi), wl.field_value(prob.truth, xb)
    ui = sol.u_int[: prep.n_int].double().cpu().numpy()
    ub = sol.u_band[: prep.n_band].double().cpu().numpy()
    d = prep.dist[prep.idx_int[: prep.n_int].long()].cpu().numpy()
    rm = lambda u, t: float(np.sqrt(np.mean((u - t) ** 2)))
    far = d >= 0.05
    near_cut = (xb[:, 0] > 0.1) & (xb[:, 0] < 0.9) & (np.abs(xb[:, 1]) < 0.05)
    out = {"workload": "slit_disk_double_sided", "ms_per_step": ms, "stage_ms": stages,
           "points_gathered": prep.n_int, "points_band": prep.n_band, "cache_points": sol.cache.n,
           "points_per_s": (prep.n_int + prep.n_band) / (ms / 1e3), "rmse_gathered": rm(ui, ti),
           "rmse_gathered_d_ge_0.05": rm(ui[far], ti[far]), "rmse_band": rm(ub, tb),
           "band_points_on_the_cut": int(near_cut.sum()),
           "band_sign_right_on_the_cut": float(np.mean(np.sign(ub[near_cut]) == np.sign(xb[near_cut, 1]))),
           "rms_truth": float(np.sqrt(np.mean(ti**2)))}
    print(json.dumps(out))


def c2screen(args):
    """The 2D step (4096-segment star) on the screened equation Lap u = sigma u
    (sigma = 4) with the plane wave exp(a.x) as data and solution: time per
    step and per stage, and the error of the gathered and band points."""
    prob = wl.problem_c2_screened(grid=args.grid)
    prep = pl.Prepared(prob, dtype="f32")
    torch.cuda.synchronize()
    for _ in range(max(1, args.warmup)):
        pl.solve(prep, with_grad=True)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(args.steps):
        sol = pl.solve(prep, with_grad=True, watch=watch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = {k: sum(v) / len(v) for k, v in watch.totals_ms().items()}
    xi = prob.eval_x[prep.idx_int[: prep.n_int].cpu().numpy()]
    xb = prob.eval_x[prep.idx_band[: prep.n_band].cpu().numpy()]
    ti, tb = wl.field_value(prob.truth, xi), wl.field_value(prob.truth, xb)
    ui = sol.u_int[: prep.n_int].double().cpu().numpy()
    ub = sol.u_band[: prep.n_band].double().cpu().numpy()
    d = prep.dist[prep.idx_int[: prep.n_int].long()].cpu().numpy()
    rm = lambda u, t: float(np.sqrt(np.mean((u - t) ** 2)))
    far = d >= 0.05
    out = {"workload": "c2screen_star4096_screened", "sigma": prob.sigma, "ms_per_step": ms, "stage_ms": stages,
           "points_gathered": prep.n_int, "points_band": prep.n_band, "cache_points": sol.cache.n,
           "points_per_s": (prep.n_int + prep.n_band) / (ms / 1e3), "rmse_gathered": rm(ui, ti),
           "rmse_gathered_d_ge_0.05": rm(ui[far], ti[far]), "rmse_band": rm(ub, tb),
           "rms_truth": float(np.sqrt(np.mean(ti**2))), "cache_walk_steps": int(sol.counters[1])}
    print(json.dumps(out))


def c3(args, prob=None):
    prob, prep = _c3_setup(args, prob)
    for w in range(args.warmup):
        pl.solve(prep, batch=100 + w, with_grad=False)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    sols = []
    ms = _time(lambda: sols.append(pl.solve(prep, batch=len(sols), with_grad=False, watch=watch)), args.steps)
    timers = {k: float(np.mean(v)) for k, v in watch.totals_ms().items()}
    stages = {k: v for k, v in timers.items() if not k.startswith("k_")}
    kernels = {k: v for k, v in timers.items() if k.startswith("k_")}
    sol = sols[-1]
    idx = prep.idx_int[: prep.n_int].cpu().numpy()
    n_box = prob.extra["n_box"]
    sub = idx[:: max(1, idx.size // 200000)]
    u = sol.u_int[: prep.n_int].double().cpu().numpy()[:: max(1, idx.size // 200000)]
    truth = wl.field_value(prob.truth, prob.eval_x[sub])
    rmse = float(np.sqrt(np.mean((u - truth) ** 2)))
    dsub = prep.dist.cpu().numpy()[sub]
    rmse_far = {f"d>={t}": float(np.sqrt(np.mean((u[dsub >= t] - truth[dsub >= t]) ** 2)))
                for t in (0.05, 0.2) if (dsub >= t).any()}
    rms_truth = float(np.sqrt(np.mean(truth**2)))
    steps = int(sol.counters[1])
    pairs = prep.n_int * sol.cache.n
    out = {"workload": prob.name, "dtype": "f32", "ms_per_step": ms,
           "points_per_s": (prep.n_int + prep.n_band) / (ms / 1e3),
           "interior_points": prep.n_int, "band_points": prep.n_band, "box_candidates": n_box,
           "slice_points": prob.extra["n_slice"], "cache_points": sol.cache.n, "walks_per_point": prob.n_walks,
           "walks": int(sol.counters[3]), "walk_steps": steps,
           "cache_walk_steps_per_s": steps / (kernels["k_walks_cache"] / 1e3),
           "kernel_ms": kernels,
           "gather_pairs_per_s": pairs / (stages["gather"] / 1e3),
           "gather_tflops_u": pairs * FLOPS_3D_BOUNDARY_U / (stages["gather"] / 1e3) / 1e12,
           "stage_ms": stages, "rmse_u_sampled": rmse, "rmse_u_far": rmse_far, "rms_u_true": rms_truth,
           "capped_walks": int(sol.counters[2]), "sigma": prob.sigma}
    print(json.dumps(out))


def c4a(args):
    prob, prep = _c3_setup(args)
    sc = prep.sc
    cache = pl.sample_cache(sc, prep.n_cand, prob.offset, prob.sides, prob.seed_cache, 0)
    W = prob.n_walks
    params = pl.walk_params(prob.eps, W, prob.seed_walks, prep.g, None, "f32")
    U, D, rec, counters = pl.cache_walks(sc, cache, params, "f32")
    nb = 81
    basis = pl.DeviceField(wl.solid_harmonics_3d(np.zeros(nb), 8))
    n = cache.n
    E = torch.empty(n, nb, dtype=torch.float64, device="cuda")
    F = torch.empty_like(E)
    t_basis = _time(lambda: B.bvc_basis_means(basis.c(), 3, n, W, B.F32, rec["exit"], rec["w1"], cache.xbar, 1,
                                              E, F))
    coefs = wl.c4_fields(64)
    coef_d = torch.from_numpy(np.ascontiguousarray(coefs)).cuda()
    nf = coefs.shape[0]
    A = torch.empty(n, nf, dtype=torch.float32, device="cuda")
    Bm = torch.empty_like(A)
    t_fields = _time(lambda: B.bvc_eval_fields(n, nb, nf, E, F, cache.w, coef_d, B.F32, A, Bm))
    cx = pl.take(cache.x, None, n, 3, n, torch.float32)
    cn = pl.take(cache.nrm, None, n, 3, n, torch.float32)
    K = prep.n_int
    xs = prep.x_int
    res = {}
    for name, prec in (("split_bf16", B.SPLIT_BF16), ("fp32", B.F32)):
        Uo = torch.empty(K, nf, dtype=torch.float32, device="cuda")
        nbytes = B.bvc_gather_multi_workspace_bytes(n, prec)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        fn = lambda: B.bvc_gather_multi(3, n, cx, cn, nf, A, Bm, K, xs, Uo, prec, ws)
        fn()
        torch.cuda.synchronize()
        res[name] = (_time(fn), Uo)
        _log(f"c4a {name} {res[name][0]:.2f} ms")
    # one plain FP32 gather of field 0, times 64 fields
    a0 = A[:, 0].contiguous()
    b0 = Bm[:, 0].contiguous()
    u0 = torch.empty(K, dtype=torch.float32, device="cuda")
    cview = dict(n=n, dtype=B.F32, x=cx, nrm=cn, a=a0, b=b0)
    t_plain = _time(lambda: B.bvc_gather_u(3, cview, None, K, xs, u0))
    # error against the closed forms on a subset of points and fields
    idx = prep.idx_int[:K].cpu().numpy()
    rng = np.random.default_rng(1)
    sub = np.sort(rng.choice(K, size=min(20000, K), replace=False))
    pts = prob.eval_x[idx[sub]]
    Ybasis = wl.real_sph_harm(8, pts)
    ls = np.array([l for l in range(9) for _ in range(2 * l + 1)])
    R = np.linalg.norm(pts, axis=1)
    basis_vals = Ybasis * R[:, None] ** ls[None, :]
    truth = basis_vals @ coefs.T  # (sub, nf)
    errs = {}
    for name in res:
        Ug = res[name][1].double().cpu().numpy()[sub]
        errs[name] = float(np.sqrt(np.mean((Ug - truth) ** 2)))
    diff = float((res["split_bf16"][1] - res["fp32"][1]).abs().max())
    pairs = K * n
    mfma_flops = 3 * 2 * K * (2 * n) * nf
    t_bf16 = res["split_bf16"][0]
    out = {"workload": "c4a_dispsphere_64fields", "fields": nf, "eval_points": K, "cache_points": n,
           "split_bf16_ms": t_bf16, "fp32_multi_ms": res["fp32"][0], "plain_fp32_x64_ms": 64 * t_plain,
           "plain_fp32_one_field_ms": t_plain,
           "field_points_per_s": {"split_bf16": K * nf / (t_bf16 / 1e3),
                                  "fp32_multi": K * nf / (res["fp32"][0] / 1e3),
                                  "plain_fp32": K * nf / (64 * t_plain / 1e3)},
           "mfma_tflops": mfma_flops / (t_bf16 / 1e3) / 1e12, "mfma_peak_bf16_tflops": 2500.0,
           "mfma_frac": mfma_flops / (t_bf16 / 1e3) / 1e12 / 2500.0,
           "generation_pairs_per_s": pairs / (t_bf16 / 1e3),
           "rmse_vs_closed_form": errs, "max_abs_split_minus_fp32": diff,
           "basis_means_ms": t_basis, "eval_fields_ms": t_fields, "walks": int(counters[3])}
    print(json.dumps(out))


def c4b(args):
    scenes = wl.c4_scenes(32)
    probs = []
    for s, (sc, nc, ne) in enumerate(scenes):
        eps = 1e-3 * sc.diagonal
        lo, hi = sc.bbox
        pts = wl.uniform_box(ne, lo, hi, wl.seed(4, 5) * 100 + s)
        g = wl.harmonic_2d(3, 1.0, 1.0)
        probs.append(wl.Problem(f"c4b_{s}", sc, g, wl.Field(), nc, 64, eps, 5 * eps, 0, pts, g, sides=2,
                                seed_walks=wl.seed(4, 4) * 100 + s, seed_cache=wl.seed(4, 3) * 100 + s))
    t = time.time()
    batch = pl.SceneBatch(probs)
    torch.cuda.synchronize()
    _log(f"c4b setup {time.time() - t:.1f}s")
    batch.launch()
    torch.cuda.synchronize()
    t_eager = _time(batch.launch, max(1, args.steps))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch.launch()
    g.replay()
    torch.cuda.synchronize()
    t_graph = _time(g.replay, max(1, args.steps))
    batch.run_sequential()
    torch.cuda.synchronize()
    t_seq = _time(batch.run_sequential, max(1, args.steps))
    n_pts = sum(e["n_int"] for e in batch.entries)
    n_cache = sum(e["cache"].n for e in batch.entries)
    pairs = sum(e["n_int"] * e["cache"].n for e in batch.entries)
    c = batch.counters()
    out = {"workload": "c4b_32_uneven_stars", "scenes": len(probs), "eval_points": n_pts, "cache_points": n_cache,
           "walks": int(c[3]), "gather_pairs": pairs, "graph_ms": t_graph, "eager_batch_ms": t_eager,
           "sequential_ms": t_seq, "points_per_s_graph": n_pts / (t_graph / 1e3),
           "points_per_s_sequential": n_pts / (t_seq / 1e3), "speedup_vs_sequential": t_seq / t_graph,
           "cache_sizes": [e["cache"].n for e in batch.entries], "eval_sizes": [e["n_int"] for e in batch.entries]}
    print(json.dumps(out))


def c2clamp(args):
    _clamp_measure(args, wl.problem_c2(), "c2clamp_star4096_poisson", with_grad=True)


def c3clamp(args):
    _clamp_measure(args, wl.problem_c3(), "c3clamp_dispsphere_laplace", with_grad=False)


def _clamp_measure(args, prob, name, with_grad):
    d = prob.scene.dim
    clamp = dict(c=args.clamp_c, n_rays=args.clamp_rays, max_hits=args.clamp_hits, seed=wl.seed(d, 7))
    t = time.time()
    plain = pl.Prepared(prob, dtype="f32")
    prep = pl.Prepared(prob, dtype="f32", clamp=clamp)
    cl = prep.clamp
    torch.cuda.synchronize()
    _log(f"{name} setup {time.time() - t:.1f}s: interior {prep.n_int}, near {cl['n_near']} "
         f"(radius {cl['radius']:.4f})")
    for _ in range(max(1, args.warmup)):
        pl.solve(prep, with_grad=with_grad)
        pl.solve(plain, with_grad=with_grad)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(args.steps):
        sol = pl.solve(prep, with_grad=with_grad, watch=watch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = {k: sum(v) / len(v) for k, v in watch.totals_ms().items()}
    watch_p = pl.Stopwatch()
    e0.record()
    for _ in range(args.steps):
        sol_p = pl.solve(plain, with_grad=with_grad, watch=watch_p)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1) / args.steps
    stages_p = {k: sum(v) / len(v) for k, v in watch_p.totals_ms().items()}
    # errors at the gathered points within reach of the correction: plain,
    # clamped only (the clamped gather over the same cache, no correction) and
    # clamped + corrected; the seeds are shared, so the three use one cache
    n = cl["n_near"]
    pos = cl["pos"][:n]
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    pts = prob.eval_x[idx_i[pos.cpu().numpy()]]
    truth = wl.field_value(prob.truth, pts)
    xs = prep.x_int[:, pos].contiguous()
    u_c = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    B.bvc_gather_u(d, sol.extra["cview"], sol.extra["sview"], n, xs, u_c, clamp=cl["c"])
    torch.cuda.synchronize()
    est = {"plain": sol_p.u_int[pos].double().cpu().numpy(), "clamped_only": u_c[:n].double().cpu().numpy(),
           "clamped_corrected": sol.u_int[pos].double().cpu().numpy()}
    err = {k: {"rmse": float(np.sqrt(np.mean((v - truth) ** 2))), "max": float(np.max(np.abs(v - truth))),
               "mean": float(np.mean(v - truth))} for k, v in est.items()}
    far = np.setdiff1d(np.arange(prep.n_int), pos.cpu().numpy())
    # beyond the clamp radius the clamp never acts: only FP32 rounding differs
    far_diff = float(np.max(np.abs(sol.u_int[: prep.n_int].double().cpu().numpy()[far]
                                   - sol_p.u_int[: prep.n_int].double().cpu().numpy()[far]))) if far.size else 0.0
    c = cl["counters"].cpu().numpy()
    out = {"workload": name, "clamp_c": cl["c"], "clamp_radius": cl["radius"],
           "n_rays": args.clamp_rays, "max_hits": args.clamp_hits, "interior_points": prep.n_int,
           "corrected_points": n, "rays": n * args.clamp_rays, "contributing_crossings": int(c[0]),
           "rays_over_capacity": int(c[1]), "correction_walks": int(c[5]), "correction_walk_steps": int(c[3]),
           "ms_per_step": ms, "ms_per_step_plain": ms_plain, "stage_ms": stages, "stage_ms_plain": stages_p,
           "error_near_offset_boundary": err, "far_points_max_abs_diff": far_diff,
           "points_per_s": (prep.n_int + prep.n_band) / (ms / 1e3)}
    print(json.dumps(out))


def c2roi(args):
    """The 2D Poisson problem with its cache on the boundary of a disk inside
    the star (Section 3.2, region of interest): the same cache size, walks and
    source count as the full step, spent on the region instead of the jagged
    boundary.  Compared with the full step on the same evaluation points."""
    prob = wl.problem_c2()
    r_in = float(np.min(np.linalg.norm(prob.scene.verts, axis=1)))
    radius = 0.6 * r_in
    t = np.linspace(0, 2 * np.pi, 1025)[:-1]
    roi = wl.Scene(2, np.stack([radius * np.cos(t), radius * np.sin(t)], 1),
                   np.array([[i, (i + 1) % 1024] for i in range(1024)], dtype=np.int32), "roi_disk")
    t0 = time.time()
    prep = pl.RoiPrepared(prob, roi, dtype="f32", n_cand=prob.n_cache)
    full = pl.Prepared(prob, dtype="f32")
    torch.cuda.synchronize()
    _log(f"c2roi setup {time.time() - t0:.1f}s: region radius {radius:.3f}, points inside {prep.n_int}")
    for _ in range(max(1, args.warmup)):
        pl.solve_roi(prep)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(args.steps):
        sol = pl.solve_roi(prep, watch=watch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = {k: sum(v) / len(v) for k, v in watch.totals_ms().items()}
    sol_full = pl.solve(full)
    torch.cuda.synchronize()
    idx = prep.idx_int[: prep.n_int].cpu().numpy()
    truth = wl.field_value(prob.truth, prob.eval_x[idx])
    u_roi = sol.u_int[: prep.n_int].double().cpu().numpy()
    # the same points in the full step (all of them are gathered there: the
    # region keeps away from the boundary band)
    pos_full = np.searchsorted(full.idx_int[: full.n_int].cpu().numpy(), idx)
    u_full = sol_full.u_int.double().cpu().numpy()[pos_full]
    rmse = lambda u: float(np.sqrt(np.mean((u - truth) ** 2)))
    out = {"workload": "c2roi_star4096_poisson_disk", "region_radius": radius, "points_inside": prep.n_int,
           "cache_points": sol.cache.n, "walks_per_point": prob.n_walks, "ms_per_step": ms, "stage_ms": stages,
           "points_per_s": prep.n_int / (ms / 1e3), "rmse_region_cache": rmse(u_roi),
           "rmse_full_cache_same_points": rmse(u_full), "rms_truth": float(np.sqrt(np.mean(truth**2))),
           "walk_steps": int(sol.counters[1])}
    print(json.dumps(out))


def c2mixed(args):
    """Boundary value caching with a Neumann part: the channel [0, 6] x [0, pi]
    (4096 segments, Dirichlet ends, reflecting walls), u = x + 0.5 e^(x-6) cos y.
    Time per step and per stage, the error of the gathered and the band
    points, and pointwise walk on stars at equal error: the per-walk variance
    at 8,192 sampled interior points gives the walks per point that reach the
    cached estimate's RMSE, and the measured walk rate converts that into
    points per second."""
    prob = wl.problem_c2_mixed(grid=args.grid)
    t0 = time.time()
    prep = pl.MixedPrepared(prob, dtype="f32")
    torch.cuda.synchronize()
    _log(f"c2mixed setup {time.time() - t0:.1f}s: gathered {prep.n_int}, band {prep.n_band}")
    for _ in range(max(1, args.warmup)):
        pl.solve_mixed(prep, with_grad=False)
    torch.cuda.synchronize()
    watch = pl.Stopwatch()
    e0, e1 = _ev(), _ev()
    e0.record()
    for _ in range(args.steps):
        sol = pl.solve_mixed(prep, with_grad=False, watch=watch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = {k: sum(v) / len(v) for k, v in watch.totals_ms().items()}
    xi = prob.eval_x[prep.idx_int[: prep.n_int].cpu().numpy()]
    xb = prob.eval_x[prep.idx_band[: prep.n_band].cpu().numpy()]
    ti, tb = wl.field_value(prob.truth, xi), wl.field_value(prob.truth, xb)
    ui = sol.u_int[: prep.n_int].double().cpu().numpy()
    ub = sol.u_band[: prep.n_band].double().cpu().numpy()
    rm = lambda u, t: float(np.sqrt(np.mean((u - t) ** 2)))
    wall = np.minimum(xi[:, 1], np.pi - xi[:, 1])
    off_wall = wall > 0.05
    err_int = rm(ui, ti)
    # pointwise walk on stars at sampled interior points
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(prep.n_int, size=min(8192, prep.n_int), replace=False))
    W = 64
    xp = torch.from_numpy(np.ascontiguousarray(xi[pick].T)).cuda()
    wp = pl.walk_params(prob.eps, W, prob.seed_walks + 7, prep.g, None, "f32")
    pl.wost(prep, wp, 1, pick.size, xp)
    torch.cuda.synchronize()
    t_pw = _time(lambda: pl.wost(prep, wp, 1, pick.size, xp), reps=3)
    U, _, cnt = pl.wost(prep, wp, 1, pick.size, xp)
    Uw = U.double().cpu().numpy().reshape(pick.size, W)
    var = float(np.mean(Uw.var(axis=1, ddof=1)))
    # pointwise walk on stars is unbiased up to the epsilon shell: its RMSE
    # with w walks per point is sqrt(var / w)
    w_eq = var / err_int**2
    walks_per_s = pick.size * W / (t_pw / 1e3)
    out = {"workload": "c2mixed_channel4096_laplace", "grid": args.grid, "points_gathered": prep.n_int,
           "points_band": prep.n_band, "cache_points": sol.cache.n, "cache_offset_points": sol.extra["n_offset"],
           "cache_candidates": prep.n_cand, "walks_per_cache_point": prob.n_walks, "ms_per_step": ms,
           "stage_ms": stages, "points_per_s": (prep.n_int + prep.n_band) / (ms / 1e3),
           "rmse_gathered": err_int, "rmse_gathered_off_walls": rm(ui[off_wall], ti[off_wall]),
           "rmse_band": rm(ub, tb), "rms_truth": float(np.sqrt(np.mean(ti**2))),
           "cache_walk_steps": int(sol.counters[1]),
           "pointwise": {"points": int(pick.size), "walks": W, "ms": t_pw, "walks_per_s": walks_per_s,
                         "mean_steps": float(cnt[1].item()) / (pick.size * W), "per_walk_variance": var,
                         "walks_for_equal_rmse": w_eq, "points_per_s_at_equal_rmse": walks_per_s / w_eq}}
    print(json.dumps(out))
