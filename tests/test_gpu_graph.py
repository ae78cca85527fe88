"""One BVC step with no host synchronisation, captured in a HIP graph
(marked gpu).

The cache sampler leaves its accepted count on the device and the walks,
means and gather read it there, so a whole solve (sampling, cache walks, FP64
means, sources, FP32 gather with the FP64 near field, band walks) enqueues
without a readback.  The device-count step must equal the host-count path
bit for bit (same cache, same streams), and a captured step must replay to
the eager result: three replays, each after unrelated eager work and a
synchronisation, each compared element by element.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import c2_like_fields, lib, small_star, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _problem(dtype="f32"):
    sc = small_star(1024)
    g, f = c2_like_fields()
    lo, hi = sc.bbox
    eps = 3e-3
    return wl.Problem("star1024_graph", sc, g, f, 4096, 32, eps, 5 * eps, 4096, wl.grid2d(128, lo, hi), g, sides=2,
                      precision=dtype, seed_walks=91, seed_cache=92, seed_sources=93)


def _outputs(prep, sol):
    out = [to_np_aos(sol.u_int, prep.n_int), to_np_aos(sol.g_int, prep.n_int), to_np_aos(sol.u_band, prep.n_band),
           to_np_aos(sol.g_band, prep.n_band)]
    n = sol.cache.n
    out += [to_np_aos(sol.uhat, n), to_np_aos(sol.dudn, n)]
    return out


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


def test_device_count_matches_host_count():
    _bvc, pl = lib()
    prob = _problem("f64")
    prep = pl.Prepared(prob)
    say(f"device count vs host count: candidates {prep.n_cand}, capacity {prep.n_cap}")
    sol = pl.solve(prep, batch=4, with_grad=True)
    torch.cuda.synchronize()
    host = pl.sample_cache(prep.sc, prep.n_cand, prob.offset, prob.sides, prob.seed_cache, 4)
    n = sol.cache.n
    assert n == host.n and 0 < n <= prep.n_cap
    for a, b in ((sol.cache.x, host.x), (sol.cache.nrm, host.nrm), (sol.cache.xbar, host.xbar)):
        assert np.array_equal(to_np_aos(a, n), to_np_aos(b, n))
    assert np.array_equal(to_np_aos(sol.cache.w, n), to_np_aos(host.w, n))
    # the same step on the host-count cache
    wp = pl.walk_params(prob.eps, prob.n_walks, prob.seed_walks, prep.g, prep.f, "f64", 4)
    U, D, _, cnt = pl.cache_walks(prep.sc, host, wp, "f64")
    uhat, dudn, a, b = pl.reduce_walks(host, prob.n_walks, U, D, "f64")
    torch.cuda.synchronize()
    assert np.array_equal(to_np_aos(sol.uhat, n), to_np_aos(uhat, n))
    assert np.array_equal(to_np_aos(sol.dudn, n), to_np_aos(dudn, n))
    assert np.array_equal(sol.counters.cpu().numpy()[1:], cnt.cpu().numpy()[1:])
    cview, sview = pl._gather_views(prep, host, a, b, 4, pl._NoWatch())
    u = torch.empty_like(sol.u_int)
    g = torch.empty_like(sol.g_int)
    _bvc.bvc_gather_grad(2, cview, sview, prep.n_int, prep.x_int, u, g)
    torch.cuda.synchronize()
    assert np.array_equal(to_np_aos(u, prep.n_int), to_np_aos(sol.u_int, prep.n_int))
    assert np.array_equal(to_np_aos(g, prep.n_int), to_np_aos(sol.g_int, prep.n_int))


def test_captured_step_replays_to_eager():
    _bvc, pl = lib()
    prob = _problem("f32")
    prep = pl.Prepared(prob)
    say(f"captured step: interior {prep.n_int}, band {prep.n_band}, capacity {prep.n_cap}")
    eager = pl.solve(prep, batch=11, with_grad=True)
    torch.cuda.synchronize()
    ref = _outputs(prep, eager)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pl.solve(prep, batch=11, with_grad=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        cap = pl.solve(prep, batch=11, with_grad=True)
    for r in range(3):
        other = pl.solve(prep, batch=20 + r, with_grad=True)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = _outputs(prep, cap)
        say(f"  replay {r}: cache {cap.cache.n} of capacity {prep.n_cap}, equal {_same(got, ref)}")
        assert cap.cache.n == eager.cache.n
        assert _same(got, ref)
        assert not np.array_equal(to_np_aos(other.u_int, prep.n_int), ref[0])
        cap.cache._n = None  # read the count again after the next replay
