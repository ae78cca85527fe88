"""GPU parity of walk on stars in 3D and with Neumann data h != 0 (2D and 3D)
against the FP64 oracle (marked gpu).

- FP64 walks walk by walk on the same Philox streams (at least 99.9% within
  1e-9; the rest may differ when an ulp flips a silhouette, crossing,
  candidate or termination decision): a box tube (Dirichlet faces x = +-1,
  reflecting y and z faces), the box with Neumann faces y = +-1 carrying
  h = -2 (u = x^2 - y^2), a dented sphere (level-2 icosphere displaced by a
  spherical-harmonic series) whose cap z > 0.3 is Neumann with h = 0.7 (folds
  of the surface as seen from inside, a Neumann / Dirichlet junction), and
  the 2D square with h = -2 on its Neumann sides; interior points, points on
  the Neumann part, offset Dirichlet points with their gradient estimate;
- FP32 walk means against the FP64 oracle's on independent streams at 3
  standard errors, as often as a normal distribution allows.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, per_walk_match, z_ok
from test_oracle_wost3 import _sh

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _dented_cap():
    sph = wl.displaced_icosphere(2, 37, amp=0.15)
    cen = sph.verts[sph.prims].mean(1)
    neu_mask = cen[:, 2] > 0.3

    def part(mask, tag):
        P = sph.prims[mask]
        used, inv = np.unique(P.ravel(), return_inverse=True)
        return wl.Scene(3, sph.verts[used], inv.reshape(P.shape).astype(np.int32), tag)

    g = wl.solid_harmonics_3d(np.random.default_rng(4).normal(0, 1, 16), 3)
    return sph, part(~neu_mask, "cap_dirichlet"), part(neu_mask, "cap_neumann"), g, wl.Field(wl.FIELD_CONST, [],
                                                                                              [0.7])


def _case(name):
    if name == "tube":
        full, d, n = wl.mixed_box((-1, -1, -1), (1, 1, 1), [False, False, True, True, True, True], 3)
        return full, d, n, _sh(lambda x: x[:, 0], 1), None
    if name == "box_h":
        full, d, n = wl.mixed_box((-1, -1, -1), (1, 1, 1), [False, False, True, True, False, False], 3)
        return full, d, n, _sh(lambda x: x[:, 0] ** 2 - x[:, 1] ** 2), wl.Field(wl.FIELD_CONST, [], [-2.0])
    if name == "dented_cap":
        return _dented_cap()
    if name == "square_h":
        full, d, n = wl.mixed_polygon([[-1, -1], [1, -1], [1, 1], [-1, 1]], [True, False, True, False],
                                      [12, 12, 12, 12], "square")
        return full, d, n, wl.harmonic_2d(2, 1.0, 0.0), wl.Field(wl.FIELD_CONST, [], [-2.0])
    raise KeyError(name)


def _interior(orc, full, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = full.bbox
    ofull = orc.Scene(full)
    out = []
    while len(out) < n:
        x = rng.uniform(lo, hi, (4 * n, full.dim))
        d, _, _ = ofull.closest(x)
        out.extend(x[(ofull.inside(x) != 0) & (d > 1e-3)])
    return np.array(out[:n])


def _run(_bvc, pl, dir_, neu, g, h, mode, x, dtype, W, seed, nrm=None, R0=None, xbar=None, eps=1e-3):
    sd, sn = pl.Scene(dir_), pl.Scene(neu)
    wp = pl.walk_params(eps, W, seed, pl.DeviceField(g), None, dtype, h=pl.DeviceField(h) if h is not None else None)
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


@pytest.mark.parametrize("name", ["tube", "box_h", "dented_cap", "square_h"])
def test_wost_interior_fp64_walk_by_walk(orc, name):
    _bvc, pl = lib()
    full, dir_, neu, g, h = _case(name)
    x = _interior(orc, full, 120, 3)
    W = 16
    say(f"wost fp64 interior {name}: {x.shape[0]} points x {W} walks")
    U, _, st, cnt = _run(_bvc, pl, dir_, neu, g, h, 1, x, "f64", W, 61)
    Uo, _, sto = orc.wost_walks(orc.Scene(dir_), orc.Scene(neu), g, orc.walk_params(1e-3, W, 61), 1, x, h=h)
    ok = per_walk_match(U, Uo)
    say(f"  match {ok.mean():.5f}, steps {st.mean():.1f}")
    assert ok.mean() >= 0.999
    assert np.mean(st == sto) >= 0.999
    assert cnt[3] == U.size and cnt[1] == st.sum()


@pytest.mark.parametrize("name", ["tube", "box_h"])
def test_wost3_boundary_and_cache_modes_fp64(orc, name):
    _bvc, pl = lib()
    say(f"wost fp64 modes 3 and 0 {name}")
    full, dir_, neu, g, h = _case(name)
    od, on, ofull = orc.Scene(dir_), orc.Scene(neu), orc.Scene(full)
    rng = np.random.default_rng(8)
    W = 16
    # points on the Neumann face y = 1 (outward +y) and y = -1 (outward -y)
    xb = np.stack([rng.uniform(-0.95, 0.95, 60), np.repeat([1.0, -1.0], 30), rng.uniform(-0.95, 0.95, 60)], 1)
    nb = np.stack([np.zeros(60), np.repeat([1.0, -1.0], 30), np.zeros(60)], 1)
    U3, _, _, _ = _run(_bvc, pl, dir_, neu, g, h, 3, xb, "f64", W, 62, nrm=nb)
    Uo3, _, _ = orc.wost_walks(od, on, g, orc.walk_params(1e-3, W, 62), 3, xb, nrm=nb, h=h)
    ok = per_walk_match(U3, Uo3)
    say(f"  mode 3 match {ok.mean():.5f}")
    assert ok.mean() >= 0.999
    # offset Dirichlet points at l = 5e-3 from the faces x = -1 and x = 1
    l = 5e-3
    xc = np.stack([np.repeat([-1 + l, 1 - l], 30), rng.uniform(-0.9, 0.9, 60), rng.uniform(-0.9, 0.9, 60)], 1)
    nc = np.stack([np.repeat([-1.0, 1.0], 30), np.zeros(60), np.zeros(60)], 1)
    R0, _, _ = ofull.closest(xc)
    _, xbar, _ = od.closest(xc)
    U0, D0, _, _ = _run(_bvc, pl, dir_, neu, g, h, 0, xc, "f64", W, 63, nrm=nc, R0=R0, xbar=xbar)
    Uo0, Do0, _ = orc.wost_walks(od, on, g, orc.walk_params(1e-3, W, 63), 0, xc, nrm=nc, R0=R0, xbar=xbar, h=h)
    okU = per_walk_match(U0, Uo0)
    # D = (dim/R0) (nu . n) (U - c) cancels when the walk exits where g equals
    # c (u = x on the face x = 1): its rounding is that of U and c, scaled
    scale = 3.0 / np.repeat(R0, W) * (1.0 + np.abs(Uo0))
    okD = np.abs(D0 - Do0) <= 1e-9 * scale
    say(f"  mode 0 match U {okU.mean():.5f} D {okD.mean():.5f}")
    assert okU.mean() >= 0.999 and okD.mean() >= 0.999


@pytest.mark.parametrize("name", ["dented_cap", "box_h", "square_h"])
def test_wost_fp32_statistical(orc, name):
    _bvc, pl = lib()
    full, dir_, neu, g, h = _case(name)
    x = _interior(orc, full, 48, 9)
    W = 256
    say(f"wost fp32 {name}")
    U, _, _, _ = _run(_bvc, pl, dir_, neu, g, h, 1, x, "f32", W, 64)
    Uo, _, _ = orc.wost_walks(orc.Scene(dir_), orc.Scene(neu), g, orc.walk_params(1e-3, W, 1064), 1, x, h=h)
    A, Bo = U.reshape(-1, W), Uo.reshape(-1, W)
    se = np.sqrt(A.var(1, ddof=1) / W + Bo.var(1, ddof=1) / W) + 1e-12
    ok, msg = z_ok(np.abs(A.mean(1) - Bo.mean(1)) / se)
    say(f"  {msg}")
    assert ok, msg
