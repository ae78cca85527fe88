"""GPU parity of walk on stars for mixed Dirichlet / Neumann boundaries (2D,
h = 0) against the FP64 oracle (marked gpu): FP64 walks walk by walk on the
same Philox streams (at least 99.9% within 1e-9; the rest may differ when an
ulp flips a silhouette, crossing or termination decision) in the three modes
(interior points, points on the Neumann part, offset Dirichlet cache points
with their gradient estimate), and FP32 walk means against the FP64 walks
(z-test); unsupported inputs are refused."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, per_walk_match
from test_oracle_wost import polygon_parts, subdivide

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


GEOMS = {
    "rectangle": (([[0, 0], [2, 0], [2, 1], [0, 1]], [True, False, True, False], 8), wl.harmonic_2d(1, 1.0, 0.0)),
    "l_shape": (([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]], [True, False, True, False, True, False], 6),
                wl.harmonic_2d(1, 1.0, 0.0)),
    "neumann_corner": (([[0, 0], [1, 0], [1, 1], [-1, 1], [-1, -1], [0, -1]],
                        [True, False, False, False, False, True], 1), wl.wedge_2d(1.0, 2.0 / 3.0)),
}


def _setup(pl, name):
    (verts, flags, k), g = GEOMS[name]
    full, dir_, neu = polygon_parts(*subdivide(verts, flags, k))
    return full, dir_, neu, g


def _interior(orc, full, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = full.bbox
    ofull = orc.Scene(full)
    out = []
    while len(out) < n:
        x = rng.uniform(lo, hi, (4 * n, 2))
        d, _, _ = ofull.closest(x)
        out.extend(x[(ofull.inside(x) != 0) & (d > 1e-3)])
    return np.array(out[:n])


def _run(_bvc, pl, dir_, neu, g, mode, x, dtype, W, seed, nrm=None, R0=None, xbar=None):
    sd, sn = pl.Scene(dir_), pl.Scene(neu)
    gd = pl.DeviceField(g)
    wp = pl.walk_params(1e-4, W, seed, gd, None, dtype)
    T = torch.float64 if dtype == "f64" else torch.float32
    n = x.shape[0]
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v.T if v.ndim == 2 else v)).to("cuda", torch.float64)
    U = torch.empty(n * W, dtype=T, device="cuda")
    D = torch.empty(n * W, dtype=T, device="cuda")
    st = torch.empty(n * W, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(_bvc.bvc_wost_workspace_bytes(sn.h), 256), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    _bvc.bvc_wost_walks(sd.h, sn.h, wp, mode, n, dev(x), dev(nrm) if nrm is not None else None,
                        dev(R0) if R0 is not None else None, dev(xbar) if xbar is not None else None, U, D, st,
                        ws, cnt)
    torch.cuda.synchronize()
    return U.double().cpu().numpy(), D.double().cpu().numpy(), st.cpu().numpy(), cnt.cpu().numpy()


@pytest.mark.parametrize("name", list(GEOMS))
def test_wost_interior_fp64_walk_by_walk(orc, name):
    _bvc, pl = lib()
    say(f"wost interior fp64 {name}")
    full, dir_, neu, g = _setup(pl, name)
    x = _interior(orc, full, 200, 3)
    W = 16
    U, _, st, cnt = _run(_bvc, pl, dir_, neu, g, 1, x, "f64", W, 21)
    Uo, _, sto = orc.wost_walks(orc.Scene(dir_), orc.Scene(neu), g, orc.walk_params(1e-4, W, 21), 1, x)
    ok = per_walk_match(U, Uo)
    say(f"  walks {U.size}: match {ok.mean():.5f}, steps {st.mean():.1f}")
    assert ok.mean() >= 0.999
    assert np.mean(st == sto) >= 0.999
    assert cnt[3] == U.size and cnt[1] == st.sum()


def test_wost_boundary_and_cache_modes_fp64(orc):
    _bvc, pl = lib()
    say("wost modes 3 and 0 fp64")
    full, dir_, neu, g = _setup(pl, "rectangle")
    od, on, ofull = orc.Scene(dir_), orc.Scene(neu), orc.Scene(full)
    rng = np.random.default_rng(5)
    W = 16
    # points on the Neumann sides (y = 0: outward -y; y = 1: outward +y)
    xb = np.stack([rng.uniform(0.05, 1.95, 60), np.repeat([0.0, 1.0], 30)], 1)
    nb = np.stack([np.zeros(60), np.repeat([-1.0, 1.0], 30)], 1)
    U3, _, _, _ = _run(_bvc, pl, dir_, neu, g, 3, xb, "f64", W, 22, nrm=nb)
    Uo3, _, _ = orc.wost_walks(od, on, g, orc.walk_params(1e-4, W, 22), 3, xb, nrm=nb)
    assert per_walk_match(U3, Uo3).mean() >= 0.999
    # offset Dirichlet points at l = 0.02 from x = 0 and x = 2
    l = 0.02
    xc = np.stack([np.repeat([l, 2 - l], 30), rng.uniform(0.1, 0.9, 60)], 1)
    nc = np.stack([np.repeat([-1.0, 1.0], 30), np.zeros(60)], 1)
    R0, _, _ = ofull.closest(xc)
    _, xbar, _ = od.closest(xc)
    U0, D0, _, _ = _run(_bvc, pl, dir_, neu, g, 0, xc, "f64", W, 23, nrm=nc, R0=R0, xbar=xbar)
    Uo0, Do0, _ = orc.wost_walks(od, on, g, orc.walk_params(1e-4, W, 23), 0, xc, nrm=nc, R0=R0, xbar=xbar)
    assert per_walk_match(U0, Uo0).mean() >= 0.999 and per_walk_match(D0, Do0).mean() >= 0.999


def test_wost_fp32_statistical(orc):
    _bvc, pl = lib()
    say("wost fp32")
    full, dir_, neu, g = _setup(pl, "neumann_corner")
    x = _interior(orc, full, 64, 7)
    W = 256
    U, _, _, _ = _run(_bvc, pl, dir_, neu, g, 1, x, "f32", W, 24)
    Uo, _, _ = orc.wost_walks(orc.Scene(dir_), orc.Scene(neu), g, orc.walk_params(1e-4, W, 24), 1, x)
    A, Bo = U.reshape(-1, W), Uo.reshape(-1, W)
    se = np.sqrt(A.var(1) / W + Bo.var(1) / W) + 1e-12
    z = (A.mean(1) - Bo.mean(1)) / se
    say(f"  max |z| {np.abs(z).max():.2f}")
    assert np.all(np.abs(z) < 5)
    exact = wl.field_value(g, x)
    zz = (A.mean(1) - exact) / (A.std(1) / np.sqrt(W) + 1e-12)
    assert np.mean(np.abs(zz) < 4) > 0.95


def test_wost_refuses_unsupported(orc):
    _bvc, pl = lib()
    say("wost unsupported")
    full, dir_, neu, g = _setup(pl, "rectangle")
    sd, sn = pl.Scene(dir_), pl.Scene(neu)
    gd = pl.DeviceField(g)
    x = torch.full((2, 4), 0.5, dtype=torch.float64, device="cuda")
    U = torch.empty(4 * 2, dtype=torch.float64, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    f = pl.DeviceField(wl.Field(1, np.zeros(0), (1.0,)))
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_wost_walks(sd.h, sn.h, pl.walk_params(1e-4, 2, 1, gd, f, "f64"), 1, 4, x, None, None, None, U,
                            None, None, ws, cnt)
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_wost_walks(sd.h, sn.h, pl.walk_params(1e-4, 2, 1, gd, None, "f64"), 2, 4, x, None, None, None, U,
                            None, None, ws, cnt)
    with pytest.raises(_bvc.BVCError):  # mode 3 needs normals
        _bvc.bvc_wost_walks(sd.h, sn.h, pl.walk_params(1e-4, 2, 1, gd, None, "f64"), 3, 4, x, None, None, None, U,
                            None, None, ws, cnt)
