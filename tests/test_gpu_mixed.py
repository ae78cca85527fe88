"""GPU parity of boundary value caching with a Neumann part (Section 3.2,
"Boundary Specification"; 2D, h = 0) against the FP64 oracle (marked gpu):
the mixed sampler's kinds bit for bit and its points, normals, weights and
distances to 1e-12; the classification of evaluation points; the whole step
in FP64 (the oracle's own cache equals the device's, walks on stars walk by
walk from the offset points, the Neumann points and the band points, the
device gather on the oracle's cache values); FP32 accuracy on the channel
workload; refused inputs."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, per_walk_match, to_np_aos
from test_oracle_wost import polygon_parts, subdivide

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


GEOMS = {
    "strip": lambda: polygon_parts(*subdivide([[0, 0], [1, 0], [1, np.pi], [0, np.pi]], [True, False, True, False], 8)),
    "l_shape": lambda: polygon_parts(*subdivide([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]],
                                                [True, False, True, False, True, False], 6)),
    "channel": lambda: wl.mixed_polygon([[0, 0], [6, 0], [6, np.pi], [0, np.pi]], [True, False, True, False],
                                        [48, 16, 48, 16], "channel_small"),
}


def _dev(v):
    return torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", torch.float64)


def _oracle_mixed_cache(ref):
    """Accepted oracle samples in the device's order: offset points, then
    Neumann points, each in index order."""
    acc, ty = ref["accept"], ref["type"]
    order = np.concatenate([np.flatnonzero(acc & (ty == 0)), np.flatnonzero(acc & (ty == 1))])
    return {k: ref[k][order] for k in ("x", "n", "w", "xbar", "R0")}, int((acc & (ty == 0)).sum())


@pytest.mark.parametrize("name", list(GEOMS))
def test_mixed_sampler_matches_oracle(orc, name):
    _bvc, pl = lib()
    say(f"mixed sampler {name}")
    full, dir_, neu = GEOMS[name]()
    sf, sd, sn = pl.Scene(full), pl.Scene(dir_), pl.Scene(neu)
    n, l = 4001, 0.07
    f64 = torch.float64
    x = torch.empty(2, n, dtype=f64, device="cuda")
    nrm, xbar = torch.empty_like(x), torch.empty_like(x)
    w = torch.empty(n, dtype=f64, device="cuda")
    R0 = torch.empty_like(w)
    kind = torch.empty(n, dtype=torch.int32, device="cuda")
    # the optional junction drop: same kinds on both sides, fewer offset points
    _bvc.bvc_sample_mixed(sf.h, sd.h, sn.h, n, l, 43, 2, x, nrm, w, xbar, R0, kind, junction_drop=0.05)
    torch.cuda.synchronize()
    ref = orc.sample_mixed(orc.Scene(full), orc.Scene(dir_), orc.Scene(neu), n, l, 43, 2, junction_drop=0.05)
    got_drop = kind.cpu().numpy()
    assert np.array_equal(got_drop, np.where(ref["accept"], ref["type"] + 1, 0))
    _bvc.bvc_sample_mixed(sf.h, sd.h, sn.h, n, l, 43, 2, x, nrm, w, xbar, R0, kind)
    torch.cuda.synchronize()
    ref = orc.sample_mixed(orc.Scene(full), orc.Scene(dir_), orc.Scene(neu), n, l, 43, 2)
    want = np.where(ref["accept"], ref["type"] + 1, 0)
    got = kind.cpu().numpy()
    say(f"  accepted {int((got > 0).sum())} of {n} ({int((got_drop > 0).sum())} with the junction drop)")
    assert np.array_equal(got, want)
    assert np.all((got_drop == got) | (got_drop == 0))
    assert np.allclose(to_np_aos(xbar), ref["xbar"], rtol=0, atol=1e-12)
    assert np.allclose(to_np_aos(x), ref["x"], rtol=0, atol=1e-12)
    assert np.allclose(to_np_aos(nrm), ref["n"], rtol=0, atol=1e-12)
    assert np.allclose(w.cpu().numpy(), ref["w"], rtol=1e-13)
    m = ref["accept"]
    assert np.allclose(R0.cpu().numpy()[m], ref["R0"][m], rtol=1e-12, atol=1e-14)
    assert np.allclose(to_np_aos(xbar)[m], ref["xbar"][m], rtol=0, atol=1e-12)


def test_mixed_classify_matches_oracle(orc):
    _bvc, pl = lib()
    say("mixed classify")
    full, dir_, neu = GEOMS["l_shape"]()
    sf, sd = pl.Scene(full), pl.Scene(dir_)
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.2, 2.2, (5000, 2))
    l = 0.1
    cls = torch.empty(x.shape[0], dtype=torch.int32, device="cuda")
    dist = torch.empty(x.shape[0], dtype=torch.float64, device="cuda")
    _bvc.bvc_classify_mixed(sf.h, sd.h, x.shape[0], _dev(x), l, cls, dist)
    torch.cuda.synchronize()
    inside = orc.Scene(full).inside(x) != 0
    dD, _, _ = orc.Scene(dir_).closest(x)
    want = np.where(~inside, 0, np.where(dD > l, 1, 2))
    assert np.array_equal(cls.cpu().numpy(), want)
    assert np.allclose(dist.cpu().numpy(), dD, rtol=1e-13, atol=1e-15)
    assert (want == 1).sum() > 1000 and (want == 2).sum() > 100


def _strip_problem(n_cand, W, eval_x, precision):
    full, dir_, neu = GEOMS["strip"]()
    g = wl.harmonic_2d(1, 0.0, 1.0)  # e^x cos y, zero flux through y = 0 and y = pi
    return wl.Problem("strip_mixed", full, g, wl.Field(), n_cand, W, 1e-4, 0.05, 0, eval_x, g, sides=1,
                      precision=precision, seed_walks=61, seed_cache=62, extra=dict(dirichlet=dir_, neumann=neu))


def test_mixed_step_fp64_matches_oracle(orc):
    _bvc, pl = lib()
    say("mixed step fp64")
    rng = np.random.default_rng(9)
    ex = np.stack([rng.uniform(0.002, 0.998, 1200), rng.uniform(0.05, np.pi - 0.05, 1200)], 1)
    prob = _strip_problem(1500, 16, ex, "f64")
    prep = pl.MixedPrepared(prob, dtype="f64", n_walks_band=8)
    sol = pl.solve_mixed(prep, with_grad=False)
    torch.cuda.synchronize()
    full, dir_, neu = prob.scene, prob.extra["dirichlet"], prob.extra["neumann"]
    of, od, on = orc.Scene(full), orc.Scene(dir_), orc.Scene(neu)
    # the oracle's own cache; the device's must be the same points
    ref = orc.sample_mixed(of, od, on, prep.n_cand, prob.offset, prob.seed_cache, 0)
    cn, n0 = _oracle_mixed_cache(ref)
    n = sol.cache.n
    assert n == cn["x"].shape[0] and sol.extra["n_offset"] == n0
    for key, t in (("x", sol.cache.x), ("n", sol.cache.nrm), ("xbar", sol.cache.xbar)):
        assert np.allclose(to_np_aos(t, n), cn[key], rtol=0, atol=1e-12), key
    # walks on stars from both parts of the cache, walk by walk
    W = prob.n_walks
    P0 = orc.walk_params(prob.eps, W, prob.seed_walks)
    U0, D0, _ = orc.wost_walks(od, on, prob.g, P0, 0, cn["x"][:n0], nrm=cn["n"][:n0], R0=cn["R0"][:n0],
                               xbar=cn["xbar"][:n0])
    P1 = orc.walk_params(prob.eps, W, prob.seed_walks, batch=pl.NEUMANN_BATCH_BIT)
    U1, _, _ = orc.wost_walks(od, on, prob.g, P1, 3, cn["x"][n0:], nrm=cn["n"][n0:])
    m0 = per_walk_match(sol.extra["U0"].cpu().numpy()[: n0 * W], U0)
    d0 = per_walk_match(sol.extra["D0"].cpu().numpy()[: n0 * W], D0)
    m1 = per_walk_match(sol.extra["U1"].cpu().numpy()[: (n - n0) * W], U1)
    say(f"  cache {n0} + {n - n0}: U-match {m0.mean():.5f} D-match {d0.mean():.5f} Neumann {m1.mean():.5f}")
    assert m0.mean() >= 0.999 and d0.mean() >= 0.999 and m1.mean() >= 0.999
    # the evaluation points split as the oracle splits them
    inside = of.inside(ex) != 0
    dD, _, _ = od.closest(ex)
    idx_i = prep.idx_int[: prep.n_int].cpu().numpy()
    idx_b = prep.idx_band[: prep.n_band].cpu().numpy()
    assert np.array_equal(idx_i, np.flatnonzero(inside & (dD > prob.offset)))
    assert np.array_equal(idx_b, np.flatnonzero(inside & (dD <= prob.offset)))
    # band walks
    Pb = orc.walk_params(prob.eps, 8, prob.seed_walks)
    Ub, _, _ = orc.wost_walks(od, on, prob.g, Pb, 1, ex[idx_b])
    mb = per_walk_match(sol.extra["Ub"].cpu().numpy()[: idx_b.size * 8], Ub)
    assert mb.mean() >= 0.999
    ub = sol.u_band.cpu().numpy()[: idx_b.size]
    okb = np.abs(ub - Ub.reshape(-1, 8).mean(1)) <= 1e-12 * (1 + np.abs(ub))
    assert okb.mean() >= 0.99
    # the oracle's means and gather; the device gather on the oracle's values
    uh, dh = orc.reduce(U0, D0, W)
    a = np.concatenate([uh, U1.reshape(-1, W).mean(1)]) * cn["w"]
    b = np.concatenate([dh, np.zeros(n - n0)]) * cn["w"]
    x = ex[idx_i]
    uo, cond = orc.gather(2, x, cn["x"], cn["n"], a, b, with_grad=False, with_cond=True)
    cview = dict(n=n, dtype=_bvc.F64, x=_dev(cn["x"]), nrm=_dev(cn["n"]), a=_dev(a), b=_dev(b))
    ug = torch.empty(x.shape[0], dtype=torch.float64, device="cuda")
    _bvc.bvc_gather_u(2, cview, None, x.shape[0], _dev(x), ug)
    torch.cuda.synchronize()
    assert np.all(np.abs(ug.cpu().numpy() - uo) <= 1e-11 * cond)
    # the device's own step lands on the oracle's estimate, both near u
    us = sol.u_int.cpu().numpy()[: prep.n_int]
    tru = wl.field_value(prob.g, x)
    e_dev, e_orc = np.sqrt(np.mean((us - tru) ** 2)), np.sqrt(np.mean((uo - tru) ** 2))
    diff = np.sqrt(np.mean((us - uo) ** 2))
    say(f"  interior {prep.n_int} band {prep.n_band}: rmse device {e_dev:.4g} oracle {e_orc:.4g} diff {diff:.3g}")
    assert diff <= 0.1 * e_orc + 1e-12


def test_mixed_channel_fp32_accuracy(orc):
    _bvc, pl = lib()
    say("mixed channel fp32")
    prob = wl.problem_c2_mixed(grid=160, n_cache=65536, n_walks=64)
    prep = pl.MixedPrepared(prob)
    sol = pl.solve_mixed(prep, with_grad=True)
    torch.cuda.synchronize()
    c = sol.counters.cpu().numpy()
    n = sol.cache.n
    assert c[3] == n * prob.n_walks and c[2] == 0
    xi = prob.eval_x[prep.idx_int[: prep.n_int].cpu().numpy()]
    xb = prob.eval_x[prep.idx_band[: prep.n_band].cpu().numpy()]
    ui = sol.u_int.double().cpu().numpy()[: prep.n_int]
    ub = sol.u_band.double().cpu().numpy()[: prep.n_band]
    ti, tb = wl.field_value(prob.g, xi), wl.field_value(prob.g, xb)
    ei, eb = np.sqrt(np.mean((ui - ti) ** 2)), np.sqrt(np.mean((ub - tb) ** 2))
    say(f"  cache {n} ({sol.extra['n_offset']} offset), interior {prep.n_int}: rmse {ei:.4g}; band {prep.n_band}: {eb:.4g}")
    scale = np.sqrt(np.mean(ti**2))
    assert ei < 0.03 * scale and eb < 0.03 * scale
    # gradient away from the walls: u = x + 0.5 e^(x-6) cos y
    gi = to_np_aos(sol.g_int, prep.n_int)
    away = (xi[:, 1] > 0.2) & (xi[:, 1] < np.pi - 0.2)
    gt = np.stack([1 + 0.5 * np.exp(xi[:, 0] - 6) * np.cos(xi[:, 1]), -0.5 * np.exp(xi[:, 0] - 6) * np.sin(xi[:, 1])], 1)
    gerr = np.sqrt(np.mean(np.sum((gi[away] - gt[away]) ** 2, 1)))
    say(f"  gradient rmse {gerr:.4g}")
    assert gerr < 0.3  # |grad u| is about 1; 5,000 cache points with 64 walks each


def test_mixed_refuses_bad_input():
    _bvc, pl = lib()
    full, dir_, neu = GEOMS["strip"]()
    sf, sd, sn = pl.Scene(full), pl.Scene(dir_), pl.Scene(neu)
    s3 = pl.Scene(wl.icosphere(1))
    f64 = torch.float64
    x = torch.empty(2, 8, dtype=f64, device="cuda")
    w = torch.empty(8, dtype=f64, device="cuda")
    k = torch.empty(8, dtype=torch.int32, device="cuda")
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_sample_mixed(sf.h, sd.h, sn.h, 8, 0.0, 1, 0, x, x, w, x, w, k)
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_sample_mixed(s3.h, sd.h, sn.h, 8, 0.1, 1, 0, x, x, w, x, w, k)
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_sample_mixed(sf.h, sd.h, sn.h, 8, 0.1, 1, 0, x, x, w, x, w, k, junction_drop=-0.1)
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_sample_mixed(sf.h, sd.h, sn.h, 8, 0.1, 1, 0, x, x, w, x, w, k, junction_drop=1.0)
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_classify_mixed(s3.h, sd.h, 8, x, 0.1, k)
    # empty inputs are no-ops
    _bvc.bvc_sample_mixed(sf.h, sd.h, sn.h, 0, 0.1, 1, 0, None, None, None, None, None, None)
    _bvc.bvc_classify_mixed(sf.h, sd.h, 0, None, 0.1, None)
    torch.cuda.synchronize()
