"""The pointwise walk entry point that allocates nothing
(bvc_pointwise_wos_noalloc, scratch in a library-owned static device array)
against bvc_pointwise_wos with caller buffers, through the C-ABI (marked gpu).

Both run the same kernels on the same Philox streams, so the means agree bit
for bit; the check is run twice in a row on one GPU, the second call with a
smaller input, so that the array's contents left by the first call cannot
leak into the second; a call beyond the array's size is refused before any
launch and leaves the outputs as they were."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import c2_like_fields, lib, small_star

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return lib()


CASES = {
    # scene, g, f, eps, walks per point, points of the two calls
    "star_poisson_f32": lambda: (small_star(), *c2_like_fields(), 3e-3, 64, "f32", (3000, 1100)),
    "star_poisson_f64": lambda: (small_star(), *c2_like_fields(), 3e-3, 32, "f64", (2100, 700)),
    "sphere_sh_f32": lambda: (wl.displaced_icosphere(3, 31), wl.solid_harmonics_3d(
        np.random.default_rng(1).normal(0, 1, 81), 8), None, 4e-3, 32, "f32", (1500, 333)),
    "sphere_sh_f64": lambda: (wl.displaced_icosphere(3, 31), wl.solid_harmonics_3d(
        np.random.default_rng(1).normal(0, 1, 81), 8), None, 4e-3, 16, "f64", (1200, 257)),
}


def _points(orc, scene, n, seed):
    lo, hi = scene.bbox
    pts = wl.uniform_box(3 * n, lo * 0.8, hi * 0.8, seed)
    pts = pts[orc.Scene(scene).inside(pts) != 0][:n]
    assert pts.shape[0] == n
    return pts


def _with_buffers(_bvc, pl, sc, params, x, with_grad):
    return pl.pointwise(sc, params, x, with_grad=with_grad)


def _noalloc(_bvc, sc, params, x, with_grad):
    d, n = x.shape
    u = torch.full((n,), float("nan"), dtype=x.dtype, device="cuda")
    g = torch.full((d, n), float("nan"), dtype=x.dtype, device="cuda") if with_grad else None
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    _bvc.bvc_pointwise_wos_noalloc(sc.h, params, n, x, u, g, cnt)
    return u, g, cnt


@pytest.mark.parametrize("case", list(CASES))
def test_noalloc_matches_pointwise_twice(B, orc, case):
    _bvc, pl = B
    scene, g, f, eps, W, dtype, sizes = CASES[case]()
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    fd = pl.DeviceField(f) if f is not None else None
    T = pl.DT[dtype]
    pts_all = _points(orc, scene, sizes[0], 7)
    for call, n in enumerate(sizes):
        for with_grad in (True, False):
            say(f"noalloc {case} call {call} n={n} W={W} grad={with_grad}")
            need = _bvc.bvc_pointwise_static_bytes(scene.dim, n, W, _bvc.dtype_code(T), with_grad)
            assert 0 < need <= _bvc.POINTWISE_STATIC_BYTES, need
            x = torch.from_numpy(np.ascontiguousarray(pts_all[:n].T)).to("cuda", T)
            params = pl.walk_params(eps, W, 500 + call, gd, fd, dtype)
            u0, g0, c0 = _with_buffers(_bvc, pl, sc, params, x, with_grad)
            u1, g1, c1 = _noalloc(_bvc, sc, params, x, with_grad)
            torch.cuda.synchronize()
            assert torch.equal(u1, u0[:n]), float((u1 - u0[:n]).abs().max())
            if with_grad:
                assert torch.equal(g1, g0[:, :n]), float((g1 - g0[:, :n]).abs().max())
            assert torch.equal(c1[1:], c0[1:]), (c1.tolist(), c0.tolist())
            assert int(c1[3]) == n * W
            assert bool(torch.isfinite(u1).all())


def test_noalloc_refuses_beyond_its_size(B, orc):
    _bvc, pl = B
    scene = small_star()
    g, f = c2_like_fields()
    sc = pl.Scene(scene)
    W = 256
    # the smallest point count whose scratch exceeds the static array
    n = 1
    while _bvc.bvc_pointwise_static_bytes(2, n, W, _bvc.F64, True) <= _bvc.POINTWISE_STATIC_BYTES:
        n *= 2
    say(f"noalloc refusal n={n} W={W}")
    x = torch.zeros(2, n, dtype=torch.float64, device="cuda")
    u = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    gr = torch.full((2, n), 7.0, dtype=torch.float64, device="cuda")
    cnt = torch.full((4,), 5, dtype=torch.int64, device="cuda")
    params = pl.walk_params(3e-3, W, 1, pl.DeviceField(g), pl.DeviceField(f), "f64")
    with pytest.raises(_bvc.BVCError) as e:
        _bvc.bvc_pointwise_wos_noalloc(sc.h, params, n, x, u, gr, cnt)
    assert e.value.code == -1 and "static" in str(e.value)
    torch.cuda.synchronize()
    assert bool((u == 7.0).all()) and bool((gr == 7.0).all()) and bool((cnt == 5).all())
    # and the entry point still works after the refusal
    m = 64
    pts = _points(orc, scene, m, 3)
    xs = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    u0, g0, _ = pl.pointwise(sc, params, xs, with_grad=True)
    u1, g1, _ = _noalloc(_bvc, sc, params, xs, True)
    torch.cuda.synchronize()
    assert torch.equal(u1, u0[:m]) and torch.equal(g1, g0[:, :m])
