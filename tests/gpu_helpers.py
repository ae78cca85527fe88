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


def cache_np(cache):
    n = cache.n
    return dict(x=to_np_aos(cache.x, n), n=to_np_aos(cache.nrm, n), w=to_np_aos(cache.w, n),
                xbar=to_np_aos(cache.xbar, n), R0=to_np_aos(cache.R0, n))


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
