"""Helpers shared by the GPU tests: run the HIP path through the C-ABI binding
and convert its [dim][n] device arrays to the oracle's (n, dim) layout."""
import numpy as np
import torch

import workloads as wl


def lib():
    from paper_2302_11825_amd import _bvc, pipeline

    return _bvc, pipeline


def to_np_aos(t, n=None):
    a = t.detach().cpu().numpy()
    if a.ndim == 1:
        return a[:n] if n is not None else a
    a = a[:, :n] if n is not None else a
    return np.ascontiguousarray(a.T).astype(np.float64)


def oracle_cache(ref, device_cache=None, atol=1e-12):
    """The oracle's own cache: the accepted candidates of an oracle sampler's
    output `ref` (all candidates with accept flags), in index order, as the
    device compacts them.  When the device's cache is given it must hold the
    same points; it is compared with the oracle's, never handed to it."""
    m = ref["accept"]
    cn = dict(x=ref["x"][m], n=ref["n"][m], w=ref["w"][m], xbar=ref["xbar"][m], R0=ref["R0"][m])
    if device_cache is not None:
        n = device_cache.n
        assert n == int(m.sum()), (n, int(m.sum()))
        for key, t in (("x", device_cache.x), ("n", device_cache.nrm), ("xbar", device_cache.xbar)):
            assert np.allclose(to_np_aos(t, n), cn[key], rtol=0, atol=atol), key
        assert np.allclose(to_np_aos(device_cache.w, n), cn["w"], rtol=1e-13, atol=0)
        assert np.allclose(to_np_aos(device_cache.R0, n), cn["R0"], rtol=1e-12, atol=atol)
    return cn


def per_walk_match(a, b, rel=1e-9):
    """|a - b| <= rel * max(|b|, s), s = RMS of b over all walks."""
    s = np.sqrt(np.mean(b * b)) + 1e-300
    return np.abs(a - b) <= rel * np.maximum(np.abs(b), s)


def small_star(n=512, seed=11, jitter="radial", sigma=0.01):
    return wl.star_polygon(n, seed, jitter=jitter, sigma=sigma)


def c2_like_fields():
    amps, centers, sigma = wl._c2_source()
    f = wl.gauss_sum(amps, centers, sigma)
    g = wl.gauss_potential_2d(amps, centers, sigma, 3, 1.0, 1.0)
    return g, f


def z_ok(z, level=3.0):
    """True when no more |z| exceed `level` than a normal distribution
    predicts: the expected count n P(|Z| > level) plus three of its Poisson
    standard deviations and one."""
    from math import erfc, sqrt

    z = np.asarray(z, dtype=np.float64)
    mu = z.size * erfc(level / sqrt(2.0))
    fails = int(np.sum(~(z < level)))
    allowed = mu + 3.0 * sqrt(mu) + 1.0
    return fails <= allowed, f"{fails} of {z.size} beyond {level} sigma (expected {mu:.2f}, allowed {allowed:.2f})"


def abs_terms(dim, ex, cy, cn, a, b, sy, sw, tau):
    """Sums of |terms| of u and of grad u per evaluation point, split into the
    pairs at r >= tau (FP32 in the kernel) and r < tau (FP64 near field)."""
    d = cy[None, :, :] - ex[:, None, :]
    r = np.linalg.norm(d, axis=2)
    nd = np.abs(np.einsum("kid,id->ki", d, cn))
    c = 2 * np.pi if dim == 2 else 4 * np.pi
    g_abs = np.abs(np.log(r)) / (2 * np.pi) if dim == 2 else 1 / (4 * np.pi * r)
    tu = np.abs(a)[None] * nd / (c * r**dim) + np.abs(b)[None] * g_abs
    tg = (4 * np.abs(a)[None] / r**dim + np.abs(b)[None] / r ** (dim - 1)) / c
    far = r >= tau * (1 - 1e-4)  # margin for the FP32 test in the kernel
    ds_ = np.linalg.norm(sy[None] - ex[:, None], axis=2)
    su = np.abs(sw)[None] * (np.abs(np.log(ds_)) / (2 * np.pi) if dim == 2 else 1 / (4 * np.pi * ds_))
    sg = np.abs(sw)[None] / (c * ds_ ** (dim - 1))
    rmin = np.minimum(np.where(far, r, np.inf).min(1), ds_.min(1))
    return ((tu * far).sum(1) + su.sum(1), (tu * ~far).sum(1), (tg * far).sum(1) + sg.sum(1),
            (tg * ~far).sum(1), rmin)


