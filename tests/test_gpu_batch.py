"""Many uneven scenes in one launch sequence (marked gpu).

The batch must reproduce, scene by scene, the single-scene call sequence on
the same caches (same walk ids and seeds, so the same walks), and a HIP graph
captured around bvc_batch_launch must give the eager result on every replay,
with other GPU work between replays.
"""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib

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
