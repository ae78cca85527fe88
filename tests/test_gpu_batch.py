"""Many uneven scenes in one launch sequence (marked gpu).

Every scene of the batch is checked against the FP64 oracle on its own
inputs: its cache equals the oracle's sampler output, the FP32 walks follow
the oracle's FP64 walks with the same ids and Philox streams walk by walk,
the cache means agree within 3 standard errors of the paired walk
differences, and u at the scene's evaluation points agrees with the oracle's
gather over its own cache and means (difference well inside the Monte Carlo
error; error against the closed form within 5% of the oracle's).  The batch
must also reproduce the single-scene call sequence, and a HIP graph captured
around bvc_batch_launch must give the eager result on every replay, with
other GPU work between replays.
"""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, oracle_cache, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _problems(n_scenes=6, seed=17):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        sc = wl.star_polygon(1024, 4100 + s)
        nc = int(round(math.exp(rng.uniform(math.log(200), math.log(2000)))))
        ne = int(round(math.exp(rng.uniform(math.log(300), math.log(6000)))))
        eps = 1e-3 * sc.diagonal
        lo, hi = sc.bbox
        pts = wl.uniform_box(ne, lo, hi, 500 + s)
        g = wl.harmonic_2d(3, 1.0, 1.0)
        out.append(wl.Problem(f"batch{s}", sc, g, wl.Field(), nc, 16, eps, 5 * eps, 0, pts, g, sides=2,
                              seed_walks=4000 + s, seed_cache=3000 + s))
    return out


def test_batch_matches_single_scene_runs():
    _bvc, pl = lib()
    say("batch vs single-scene runs")
    B = pl.SceneBatch(_problems())
    B.launch()
    torch.cuda.synchronize()
    seq = B.run_sequential()
    torch.cuda.synchronize()
    total_walks = 0
    for e, us in zip(B.entries, seq):
        n = e["n_int"]
        ub = e["u"][:n].double().cpu().numpy()
        uo = us[:n].double().cpu().numpy()
        scale = np.abs(uo).max() + 1e-30
        assert np.allclose(ub, uo, rtol=1e-5, atol=1e-6 * scale), e["problem"].name
        total_walks += e["cache"].n * e["problem"].n_walks
    c = B.counters()
    assert int(c[3]) == total_walks and int(c[0]) >= total_walks


def test_batch_matches_oracle(orc):
    """Each scene of one batch launch against the oracle (Algorithm 1 per
    scene: cache walks, means, gather)."""
    _bvc, pl = lib()
    probs = _problems(4, seed=29)
    say("batch vs oracle: " + ", ".join(f"{p.name} n_cache {p.n_cache} n_eval {p.eval_x.shape[0]}" for p in probs))
    B = pl.SceneBatch(probs)
    B.launch()
    torch.cuda.synchronize()
    res = B.results()
    for e, (Ug, Dg, ag, bg) in zip(B.entries, res):
        p, cache = e["problem"], e["cache"]
        W, n = p.n_walks, cache.n
        osc = orc.Scene(p.scene)
        cn = oracle_cache(osc.sample_cache(cache.n_candidates, p.offset, p.sides, p.seed_cache, 0), cache)
        ref = orc.cache_walks(osc, p.g, None, orc.walk_params(p.eps, W, p.seed_walks), cn)
        Ug = Ug.double().cpu().numpy()
        Dg = Dg.double().cpu().numpy()
        # walk by walk: the same ids and streams give the same walks up to
        # FP32 rounding, except where rounding flips a termination or
        # closest-primitive decision
        for A, Bo, name in ((Ug, ref["U"], "U"), (Dg, ref["D"], "D")):
            s_ = np.sqrt(np.mean(Bo**2))
            agree = np.abs(A - Bo) <= 1e-3 * np.maximum(np.abs(Bo), s_)
            say(f"{p.name} {name}: {agree.mean():.4f} of {A.size} walks agree")
            assert agree.mean() >= 0.97, (p.name, name, agree.mean())
        # cache means: paired differences of the W walks of each point
        for A, Bo, got in ((Ug, ref["U"], ag), (Dg, ref["D"], bg)):
            dlt = (A - Bo).reshape(n, W)
            scale = np.sqrt(np.mean(Bo**2))
            se = np.sqrt(dlt.var(1) / W) + 1e-5 * scale
            z = np.abs(dlt.mean(1)) / se
            assert np.mean(z < 3.0) >= 0.99, (p.name, np.mean(z < 3.0))
            # the stored cache values are the FP64 means of the device's own
            # walks times w, rounded once to FP32
            mean_g = A.reshape(n, W).mean(1) * cn["w"]
            assert np.allclose(got.double().cpu().numpy(), mean_g, rtol=2e-6, atol=1e-7 * np.abs(mean_g).max())
        # u at the scene's interior points against the oracle's own chain
        cls = osc.classify(p.eval_x, p.offset)
        idx_o = np.flatnonzero(cls == 1)
        assert np.array_equal(e["idx"][: e["n_int"]].cpu().numpy(), idx_o)
        uh, dh = orc.reduce(ref["U"], ref["D"], W)
        pts = p.eval_x[idx_o]
        uo = orc.gather(2, pts, cn["x"], cn["n"], uh * cn["w"], dh * cn["w"], with_grad=False)
        ub = e["u"][: e["n_int"]].double().cpu().numpy()
        truth = wl.field_value(p.g, pts)
        err_o = np.sqrt(np.mean((uo - truth) ** 2))
        err_b = np.sqrt(np.mean((ub - truth) ** 2))
        diff = np.sqrt(np.mean((ub - uo) ** 2))
        say(f"{p.name}: rmse oracle {err_o:.4g} batch {err_b:.4g} rms(batch - oracle) {diff:.3g}")
        assert diff <= 0.1 * err_o, (p.name, diff, err_o)
        assert abs(err_b - err_o) <= 0.05 * err_o, (p.name, err_b, err_o)


def test_batch_graph_replays_match_eager():
    _bvc, pl = lib()
    say("batch graph capture and replay")
    B = pl.SceneBatch(_problems(5, seed=23))
    B.launch()
    torch.cuda.synchronize()
    ref = [e["u"][: e["n_int"]].clone() for e in B.entries]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.launch()  # warm on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        B.launch()
    for rep in range(3):
        for e in B.entries:
            e["u"].fill_(float("nan"))
        B.run_sequential()  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, r in zip(B.entries, ref):
            assert torch.equal(e["u"][: e["n_int"]], r), (rep, e["problem"].name)
