"""Differentiable inverse problem (marked gpu): boundary data given by 256
Fourier coefficients on the star domain, 4096 noisy interior observations,
gradient descent through the hand-written adjoints of the gather and the
cache (walks fixed, read back from their exit records).

Checks:
  - the adjoint gradient of the FP32 forward against the FP64 oracle gradient
    on the same exit records (relative 1e-3);
  - central finite differences (step 1e-4) of the FP64 forward along 16 random
    directions of theta (the loss is quadratic in theta, so central
    differences are exact up to rounding: 1e-7) and of the evaluation
    positions (1e-3, points at least 0.05 from the boundary);
  - gradient descent lowers the loss by two orders of magnitude and recovers
    the low-order coefficients.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def inv(orc):
    _bvc, pl = lib()
    from paper_2302_11825_amd import autograd as ag

    p = wl.problem_c5()
    say("inverse setup: walks and basis means")
    sc = pl.Scene(p["scene"])
    l, eps, W = p["offset"], p["eps"], p["n_walks"]
    n_cand = pl.candidates_for(sc, p["n_cache"], l, 2, p["seed_cache"])
    cache = pl.sample_cache(sc, n_cand, l, 2, p["seed_cache"])
    g = pl.DeviceField(wl.fourier_2d(p["theta_true"]))
    U, D, rec, _ = pl.cache_walks(sc, cache, pl.walk_params(eps, W, p["seed_walks"], g, None, "f32"), "f32")
    basis = pl.DeviceField(wl.fourier_2d(np.zeros(256)))
    n = cache.n
    E = torch.empty(n, 256, dtype=torch.float64, device="cuda")
    F = torch.empty_like(E)
    _bvc.bvc_basis_means(basis.c(), 2, n, W, _bvc.F32, rec["exit"], rec["w1"], cache.xbar, 1, E, F)
    obs64 = torch.from_numpy(np.ascontiguousarray(p["obs_candidates"].T)).cuda()
    cls, dist = pl.classify(sc, obs64, l)
    idx, cnt = sc.compact(cls, 1)
    k = min(4096, cnt)
    x32 = pl.take(obs64, idx, k, 2, obs64.shape[1], torch.float32)
    x64 = pl.take(obs64, idx, k, 2, obs64.shape[1], torch.float64)
    d_obs = pl.take(dist, idx, k, 1, dist.shape[0], torch.float64)
    cx32 = pl.take(cache.x, None, n, 2, n, torch.float32)
    cn32 = pl.take(cache.nrm, None, n, 2, n, torch.float32)
    torch.cuda.synchronize()
    theta_true = torch.from_numpy(p["theta_true"]).cuda()
    with torch.no_grad():
        a, b = ag.cache_values(theta_true, E, F, cache.w, torch.float32)
        u_clean = ag.gather(a, b, x32, cx32, cn32)
    noise = torch.from_numpy(np.random.default_rng(p["noise_seed"]).normal(0, p["noise_sigma"], k)).cuda()
    u_obs = (u_clean.double() + noise).float()
    return dict(p=p, sc=sc, cache=cache, rec=rec, E=E, F=F, x32=x32, x64=x64, d_obs=d_obs, cx32=cx32,
                cn32=cn32, u_obs=u_obs, theta_true=theta_true, n=n, k=k, W=W, ag=ag, pl=pl)


def _loss(I, theta, dtype=torch.float32, x=None):
    ag = I["ag"]
    c = I["cache"]
    if dtype == torch.float64:
        cx, cn, xx = c.x, c.nrm, (I["x64"] if x is None else x)
    else:
        cx, cn, xx = I["cx32"], I["cn32"], (I["x32"] if x is None else x)
    a, b = ag.cache_values(theta, I["E"], I["F"], c.w, dtype)
    u = ag.gather(a, b, xx, cx, cn)
    r = u - I["u_obs"].to(dtype)
    return 0.5 * (r * r).sum()


def test_adjoint_matches_oracle_gradient(inv, orc):
    I = inv
    say("inverse: adjoint vs oracle gradient")
    theta = torch.zeros(256, dtype=torch.float64, device="cuda", requires_grad=True)
    L = _loss(I, theta)
    L.backward()
    g_gpu = theta.grad.cpu().numpy()
    # oracle: its own basis means from the same exit records, FP64 throughout
    n, W = I["n"], I["W"]
    exit_pts = to_np_aos(I["rec"]["exit"], n * W)
    w1 = I["rec"]["w1"].double().cpu().numpy()[: n * W]
    xbar = to_np_aos(I["cache"].xbar, n)
    Eo, Fo = orc.basis_means(wl.fourier_2d(np.zeros(256)), 2, exit_pts, w1, xbar, W)
    w = I["cache"].w.cpu().numpy()[:n]
    cy, cn = to_np_aos(I["cx32"], n), to_np_aos(I["cn32"], n)
    x = to_np_aos(I["x32"], I["k"])
    a = w * (Eo @ np.zeros(256))
    b = w * (Fo @ np.zeros(256))
    u = orc.gather(2, x, cy, cn, a, b, with_grad=False)
    r = u - I["u_obs"].double().cpu().numpy()
    da, db, _, _ = orc.gather_backward(2, x, r, cy, cn, a, b)
    g_ref = Eo.T @ (w * da) + Fo.T @ (w * db)
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    say(f"  relative gradient error {rel:.2e}")
    assert rel < 1e-3


def test_finite_differences_theta_and_positions(inv):
    I = inv
    say("inverse: finite differences")
    rng = np.random.default_rng(9)
    theta0 = torch.from_numpy(rng.normal(0, 0.1, 256)).cuda()
    th = theta0.clone().requires_grad_(True)
    L = _loss(I, th, torch.float64)
    L.backward()
    g = th.grad.clone()
    h = 1e-4
    for _ in range(16):
        v = torch.from_numpy(rng.normal(0, 1, 256)).cuda()
        with torch.no_grad():
            fd = (_loss(I, theta0 + h * v, torch.float64) - _loss(I, theta0 - h * v, torch.float64)) / (2 * h)
        an = (g * v).sum()
        assert abs(float(fd - an)) <= 1e-7 * (abs(float(an)) + float(L)), (float(fd), float(an))
    # positions: only points at least 0.05 from the boundary are moved
    x = I["x64"].clone().requires_grad_(True)
    L = _loss(I, theta0, torch.float64, x)
    L.backward()
    gx = x.grad.clone()
    far = (I["d_obs"][: I["k"]] >= 0.05).double()
    for _ in range(16):
        v = torch.from_numpy(rng.normal(0, 1, (2, I["k"]))).cuda() * far
        with torch.no_grad():
            fd = (_loss(I, theta0, torch.float64, I["x64"] + h * v)
                  - _loss(I, theta0, torch.float64, I["x64"] - h * v)) / (2 * h)
        an = (gx * v).sum()
        assert abs(float(fd - an)) <= 1e-3 * abs(float(an)) + 1e-9, (float(fd), float(an))


def test_gradient_descent_recovers_boundary_data(inv):
    I = inv
    say("inverse: gradient descent")
    # step size from the largest eigenvalue of J^T J (power iteration through the adjoints)
    v = torch.ones(256, dtype=torch.float64, device="cuda") / 16
    zero = torch.zeros(256, dtype=torch.float64, device="cuda")
    with torch.no_grad():
        L0 = float(_loss(I, zero))
    lam = 1.0
    for _ in range(15):
        th = v.clone().requires_grad_(True)
        a, b = I["ag"].cache_values(th, I["E"], I["F"], I["cache"].w, torch.float32)
        u = I["ag"].gather(a, b, I["x32"], I["cx32"], I["cn32"])
        (0.5 * (u * u).sum()).backward()
        jtjv = th.grad
        lam = float(jtjv.norm() / v.norm())
        v = jtjv / jtjv.norm()
    step = 1.0 / lam
    theta = torch.zeros(256, dtype=torch.float64, device="cuda")
    prev = theta.clone()
    for it in range(400):
        y = theta + (it / (it + 3)) * (theta - prev)
        y = y.detach().requires_grad_(True)
        L = _loss(I, y)
        L.backward()
        prev = theta
        theta = (y - step * y.grad).detach()
    with torch.no_grad():
        L1 = float(_loss(I, theta))
    low = slice(0, 9)
    err = float((theta[low] - I["theta_true"][low]).norm() / I["theta_true"][low].norm())
    say(f"  loss {L0:.3e} -> {L1:.3e}, low-order coefficient error {err:.3f}")
    assert L1 < 1e-2 * L0
    assert err < 0.1
