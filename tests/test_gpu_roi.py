"""GPU parity of the region-of-interest cache (Section 3.2, "Boundary
Specification") against the FP64 oracle (marked gpu): the sampler's accept
flags bit for bit and its points, normals, weights and domain distances to
1e-13 (2D and 3D); the classification of evaluation points against the
region; and the whole ROI step in FP64 against the oracle's own cache, walks, means
and gather, plus its accuracy inside the region."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, oracle_cache, per_walk_match, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def shifted(scene, scale, shift):
    return wl.Scene(scene.dim, scene.verts * scale + np.asarray(shift)[None], scene.prims, scene.name + "_roi")


CASES = {
    "2d": lambda: (wl.circle_polygon(256), shifted(wl.circle_polygon(128), 0.4, (0.2, -0.1))),
    "2d_partly_outside": lambda: (wl.circle_polygon(256), shifted(wl.circle_polygon(64), 0.5, (0.8, 0.0))),
    "3d": lambda: (wl.icosphere(3), shifted(wl.icosphere(2), 0.45, (0.1, 0.05, -0.2))),
}


@pytest.mark.parametrize("case", list(CASES))
def test_roi_sampler_matches_oracle(orc, case):
    _bvc, pl = lib()
    dom, roi = CASES[case]()
    say(f"roi sampler {case}")
    sd, sr = pl.Scene(dom), pl.Scene(roi)
    d, n = dom.dim, 3001
    f64 = torch.float64
    x = torch.empty(d, n, dtype=f64, device="cuda")
    nrm, xbar = torch.empty_like(x), torch.empty_like(x)
    w = torch.empty(n, dtype=f64, device="cuda")
    R0 = torch.empty_like(w)
    acc = torch.empty(n, dtype=torch.int32, device="cuda")
    _bvc.bvc_sample_roi(sd.h, sr.h, n, 41, 3, x, nrm, w, xbar, R0, acc)
    torch.cuda.synchronize()
    ref = orc.sample_roi(orc.Scene(dom), orc.Scene(roi), n, 41, 3)
    assert np.array_equal(acc.cpu().numpy().astype(bool), ref["accept"])
    assert np.allclose(to_np_aos(x), ref["x"], rtol=0, atol=1e-13)
    assert np.allclose(to_np_aos(nrm), ref["n"], rtol=0, atol=1e-13)
    assert np.allclose(w.cpu().numpy(), ref["w"], rtol=1e-13)
    m = ref["accept"]
    assert np.allclose(R0.cpu().numpy()[m], ref["R0"][m], rtol=1e-12, atol=1e-15)
    assert np.allclose(to_np_aos(xbar)[m], ref["xbar"][m], rtol=0, atol=1e-13)


def test_roi_step_fp64_matches_oracle(orc):
    _bvc, pl = lib()
    say("roi step fp64")
    dom, roi = CASES["2d"]()
    g = wl.harmonic_2d(3, 1.0, 1.0)
    rng = np.random.default_rng(8)
    ex = rng.uniform(-0.7, 0.7, (1500, 2))
    prob = wl.Problem("roi_disk", dom, g, wl.Field(), 1200, 32, 1e-4, 1e-4, 0, ex, g, sides=1, precision="f64",
                      seed_walks=91, seed_cache=92)
    prep = pl.RoiPrepared(prob, roi, dtype="f64")
    sol = pl.solve_roi(prep, with_grad=True)
    torch.cuda.synchronize()
    # evaluation points: exactly those inside the region
    idx = np.flatnonzero(orc.Scene(roi).classify(ex, 0.0) == 1)
    assert np.array_equal(prep.idx_int[: prep.n_int].cpu().numpy(), idx)
    # the oracle's own cache (equal to the device's), its walks, means and gather
    cn = oracle_cache(orc.sample_roi(orc.Scene(dom), orc.Scene(roi), prep.n_cand, prob.seed_cache, 0), sol.cache)
    W = prob.n_walks
    ref = orc.cache_walks(orc.Scene(dom), g, None, orc.walk_params(prob.eps, W, prob.seed_walks), cn)
    n = sol.cache.n
    assert per_walk_match(sol.extra["U"].cpu().numpy()[: n * W], ref["U"]).mean() >= 0.999
    uh, dh = orc.reduce(ref["U"], ref["D"], W)
    a, b = uh * cn["w"], dh * cn["w"]
    x = ex[idx]
    uo, go, cond = orc.gather(2, x, cn["x"], cn["n"], a, b, with_grad=True, with_cond=True)
    ug = sol.u_int.cpu().numpy()[: prep.n_int]
    ok = np.abs(ug - uo) <= 1e-9 * (np.abs(uo) + cond)
    assert ok.mean() >= 0.99
    # and the estimate is close to the solution inside the region
    err = np.sqrt(np.mean((ug - wl.field_value(g, x)) ** 2))
    say(f"  inside {prep.n_int}: rmse {err:.4g}")
    assert err < 0.03 * np.sqrt(np.mean(wl.field_value(g, x) ** 2))
