"""The band walks of a step run on a second stream beside the cache walks
(marked gpu).  Every walk keeps its id and random stream, so the results may
not depend on which of the two walk launches starts first, on steps issued
back to back without a synchronisation, or on the overlap itself: the
overlapped band walks must equal the same pointwise walks run alone, bit for
bit.  The mixed step (walks on stars, band walks with a workspace of their
own) is held to the same rule.
"""
import sys

import numpy as np
import torch

from gpu_helpers import lib, to_np_aos
from test_gpu_graph import _outputs, _problem, _same
from test_gpu_mixed import _strip_problem

import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_band_walks_beside_cache_walks_either_order():
    _bvc, pl = lib()
    prob = _problem("f32")
    prep = pl.Prepared(prob)
    nb = prep.n_band
    say(f"overlapped band walks: {prep.n_int} gathered, {nb} band points")
    assert nb > 0
    sols = []
    for first in (True, False, True):
        # issued back to back: no synchronisation between the steps
        prep.band_first = first
        sols.append(pl.solve(prep, batch=3, with_grad=True))
    torch.cuda.synchronize()
    outs = [_outputs(prep, s) for s in sols]
    assert _same(outs[0], outs[1]) and _same(outs[0], outs[2])
    for s in sols[1:]:
        assert torch.equal(s.pw_counters, sols[0].pw_counters) and torch.equal(s.counters, sols[0].counters)
    # the same band walks alone on the current stream
    wpb = pl.walk_params(prob.eps, prob.n_walks, prob.seed_walks, prep.g, prep.f, "f32", 3, sigma=prob.sigma,
                         side_read=prob.side_read)
    u, g, _ = pl.pointwise(prep.sc, wpb, prep.x_band[:, :nb], True, order=prep.band_order)
    torch.cuda.synchronize()
    assert np.array_equal(to_np_aos(u, nb), to_np_aos(sols[0].u_band, nb))
    assert np.array_equal(to_np_aos(g, nb), to_np_aos(sols[0].g_band, nb))


def test_mixed_band_walks_overlapped():
    _bvc, pl = lib()
    rng = np.random.default_rng(19)
    ex = np.stack([rng.uniform(0.002, 0.998, 2000), rng.uniform(0.05, np.pi - 0.05, 2000)], 1)
    prob = _strip_problem(1500, 16, ex, "f32")
    prep = pl.MixedPrepared(prob, n_walks_band=8)
    nb = prep.n_band
    say(f"mixed step, overlapped band walks: {prep.n_int} gathered, {nb} band points")
    assert nb > 0
    a = pl.solve_mixed(prep, batch=2, with_grad=False)
    b = pl.solve_mixed(prep, batch=2, with_grad=False)
    torch.cuda.synchronize()
    c = pl.solve_mixed(prep, batch=2, with_grad=False)
    torch.cuda.synchronize()
    for s in (b, c):
        assert np.array_equal(to_np_aos(s.u_band, nb), to_np_aos(a.u_band, nb))
        assert np.array_equal(to_np_aos(s.u_int, prep.n_int), to_np_aos(a.u_int, prep.n_int))
        assert torch.equal(s.pw_counters, a.pw_counters)
    # the band walks alone, in sequence on the current stream
    wpb = pl.walk_params(prob.eps, prep.W_band, prob.seed_walks, prep.g, None, "f32", 2, side_read=prob.side_read)
    Ub, _, _ = pl.wost(prep, wpb, 1, nb, prep.x_band, dtype="f32")
    torch.cuda.synchronize()
    assert torch.equal(Ub[: nb * prep.W_band], a.extra["Ub"][: nb * prep.W_band])
