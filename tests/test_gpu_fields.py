"""Boundary data evaluated by the walks' finishing kernel (marked gpu): FP32
walks read solid-harmonic data through an FP32 table of coefficient times
normalisation; the values at the walks' exits are compared with the FP64
oracle's series."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_helpers import lib

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L", [3, 8, 16])
def test_fp32_solid_harmonics_at_exits(orc, L):
    """FP32 walks read solid-harmonic boundary data from an FP32 table of
    coefficient times normalisation: for Laplace cache walks U is g at the
    exit, compared at 64 exits with the FP64 oracle's series within a few ulp
    per degree of the sum of |terms|."""
    _bvc, pl = lib()
    say(f"fp32 solid harmonics L={L}")
    scene = wl.displaced_icosphere(3, 31)
    coef = np.random.default_rng(L).normal(0, 1, (L + 1) ** 2)
    g = wl.solid_harmonics_3d(coef, L)
    sc = pl.Scene(scene)
    gd = pl.DeviceField(g)
    cache = pl.sample_cache(sc, 2000, 2e-2, 1, 4, 0)
    W = 4
    U, D, rec, _ = pl.cache_walks(sc, cache, pl.walk_params(4e-3, W, 21, gd, None, "f32"), "f32")
    torch.cuda.synchronize()
    k = cache.n * W
    sel = np.linspace(0, k - 1, 64).astype(int)
    ex = rec["exit"][:, :k].double().cpu().numpy().T[sel]
    u = U[:k].double().cpu().numpy()[sel]
    ref = orc.field_eval(g, ex)
    S = np.zeros(len(sel))
    for b in range((L + 1) ** 2):
        S += np.abs(coef[b] * orc.basis_eval(g, 3, b, ex))
    tol = (L + 4) * 2.0**-22 * S
    err = np.abs(u - ref)
    say(f"  max err / tol {np.max(err / tol):.3f}")
    assert np.all(err <= tol)
