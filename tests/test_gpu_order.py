"""Launch order of the walks (marked gpu): bvc_spatial_order lists the points
0..count-1 once each (count from the host or from a device count), and walks
started in that order reproduce the walks started in point order bit for bit,
since every walk keeps its id, random stream and record slot.  An order entry
outside the live points skips that point's walks and nothing else."""
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


def _scene_fields(dim):
    if dim == 2:
        g, f = c2_like_fields()
        return small_star(), g, f, 1.5e-2, 2, 3e-3
    scene = wl.displaced_icosphere(3, 31)
    g = wl.solid_harmonics_3d(np.random.default_rng(1).normal(0, 1, 16), 3)
    return scene, g, None, 2e-2, 1, 4e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_spatial_order_is_a_permutation(dim):
    _bvc, pl = lib()
    say(f"spatial order permutation dim={dim}")
    scene = _scene_fields(dim)[0]
    sc = pl.Scene(scene)
    rng = np.random.default_rng(5 + dim)
    for n in (1, 255, 4097):
        x = rng.uniform(-1.5, 1.5, (dim, n))
        x[:, 0] = np.nan  # a point that is not finite falls in an edge cell
        for T in (torch.float64, torch.float32):
            xd = torch.from_numpy(x).to("cuda", T)
            o = sc.spatial_order(xd, n).cpu().numpy()
            assert np.array_equal(np.sort(o), np.arange(n))
    # a device count orders the first count points only
    n, cnt = 3000, 1234
    x = torch.from_numpy(rng.uniform(-1, 1, (dim, n))).to("cuda", torch.float64)
    n_dev = torch.tensor([cnt], dtype=torch.int64, device="cuda")
    o = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    work = sc.order_work()
    _bvc.bvc_spatial_order(sc.h, n, x, o, work, n_dev=n_dev)
    o = o.cpu().numpy()
    assert np.array_equal(np.sort(o[:cnt]), np.arange(cnt)) and np.all(o[cnt:] == -7)
    # the order follows the cells: consecutive entries lie close on average
    xs = x.cpu().numpy()[:, o[:cnt]]
    step = np.linalg.norm(np.diff(xs, axis=1), axis=0).mean()
    rand = np.linalg.norm(np.diff(x.cpu().numpy()[:, :cnt], axis=1), axis=0).mean()
    say(f"  mean step ordered {step:.3f}, in point order {rand:.3f}")
    assert step < 0.5 * rand


@pytest.mark.parametrize("dim", [2, 3])
def test_ordered_cache_walks_are_bit_identical(dim):
    _bvc, pl = lib()
    say(f"ordered cache walks dim={dim}")
    scene, g, f, l, sides, eps = _scene_fields(dim)
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    fd = pl.DeviceField(f) if f is not None else None
    W = 32
    # device count below the capacity, as the timed step samples it
    cache = pl.sample_cache_device(sc, 5000, 5000, l, sides, 9, 0)
    n, cnt = cache.cap, cache.n
    params = pl.walk_params(eps, W, 77, gd, fd, "f32")
    # (these trees fit L2, where the pipeline keeps point order: set it here)
    cache.order = sc.spatial_order(cache.x, n, cache.n_dev)
    U1, D1, rec1, c1 = pl.cache_walks(sc, cache, params, "f32")
    # the same walks in point order
    p0 = pl.walk_params(eps, W, 77, gd, fd, "f32")
    p0.n_dev = cache.n_dev.data_ptr()
    U0, D0 = torch.empty_like(U1), torch.empty_like(D1)
    ex0, w0 = torch.empty_like(rec1["exit"]), torch.empty_like(rec1["w1"])
    c0 = torch.zeros(4, dtype=torch.int64, device="cuda")
    _bvc.bvc_cache_walks(sc.h, p0, n, cache.x, cache.nrm, cache.R0, cache.xbar, U0, D0, ex0, w0, None, c0)
    torch.cuda.synchronize()
    k = cnt * W
    assert torch.equal(U1[:k], U0[:k]) and torch.equal(D1[:k], D0[:k])
    assert torch.equal(rec1["exit"][:, :k], ex0[:, :k]) and torch.equal(rec1["w1"][:k], w0[:k])
    assert torch.equal(c1[1:], c0[1:]) and int(c1[3]) == k
    # an entry outside the live points skips that point's walks
    bad = cache.order.clone()
    victim = int(bad[cnt // 2])
    bad[cnt // 2] = cnt + 5 if cnt + 5 < n else -1
    p2 = pl.walk_params(eps, W, 77, gd, fd, "f32")
    p2.n_dev = cache.n_dev.data_ptr()
    p2.order = bad.data_ptr()
    U2 = torch.full_like(U1, float("nan"))
    D2, ex2, w2 = torch.empty_like(D1), torch.empty_like(ex0), torch.empty_like(w0)
    c2 = torch.zeros(4, dtype=torch.int64, device="cuda")
    _bvc.bvc_cache_walks(sc.h, p2, n, cache.x, cache.nrm, cache.R0, cache.xbar, U2, D2, ex2, w2, None, c2)
    torch.cuda.synchronize()
    skip = torch.zeros(n * W, dtype=torch.bool, device="cuda")
    skip[victim * W:(victim + 1) * W] = True
    assert torch.isnan(U2[:k][skip[:k]]).all()
    assert torch.equal(U2[:k][~skip[:k]], U0[:k][~skip[:k]])
    assert int(c2[3]) == k - W


@pytest.mark.parametrize("dim", [2, 3])
def test_ordered_pointwise_walks_are_bit_identical(dim):
    _bvc, pl = lib()
    say(f"ordered pointwise walks dim={dim}")
    scene, g, f, l, sides, eps = _scene_fields(dim)
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    fd = pl.DeviceField(f) if f is not None else None
    rng = np.random.default_rng(40 + dim)
    m = 2000
    x = rng.uniform(-0.6, 0.6, (dim, m))
    cls, _ = pl.classify(sc, torch.from_numpy(x).cuda(), l)
    keep = cls.cpu().numpy() != 0
    xd = torch.from_numpy(np.ascontiguousarray(x[:, keep])).to("cuda", torch.float32)
    nk = xd.shape[1]
    order = sc.spatial_order(xd, nk)
    u0, g0, c0 = pl.pointwise(sc, pl.walk_params(eps, 16, 3, gd, fd, "f32"), xd, True)
    u1, g1, c1 = pl.pointwise(sc, pl.walk_params(eps, 16, 3, gd, fd, "f32"), xd, True, order=order)
    torch.cuda.synchronize()
    say(f"  {nk} points")
    assert torch.equal(u1[:nk], u0[:nk]) and torch.equal(g1[:, :nk], g0[:, :nk])
    assert torch.equal(c1[1:], c0[1:])


def test_order_refused_where_not_taken():
    """The clamp correction's walks run from a queue of ids and take no launch
    order."""
    _bvc, pl = lib()
    say("order refused by the clamp correction")
    g, f = c2_like_fields()
    sc = pl.Scene(small_star())
    gd = pl.DeviceField(g)
    p = pl.walk_params(3e-3, 1, 5, gd, None, "f32")
    order = torch.zeros(4, dtype=torch.int32, device="cuda")
    p.order = order.data_ptr()
    cp = _bvc.clamp_params(1.5e-2, 2, 20.0, 4, 2)
    x = torch.zeros(2, 1, dtype=torch.float64, device="cuda")
    wind = torch.zeros(1, dtype=torch.int32, device="cuda")
    pos = torch.zeros(1, dtype=torch.int64, device="cuda")
    u = torch.zeros(1, dtype=torch.float32, device="cuda")
    nbytes = _bvc.bvc_clamp_workspace_bytes(2, _bvc.F32, 1, 4, 2)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(6, dtype=torch.int64, device="cuda")
    with pytest.raises(_bvc.BVCError):
        _bvc.bvc_clamp_correction(sc.h, p, cp, 1, x, wind, pos, u, ws, cnt)

