"""Multi-RHS gather parity (marked gpu): FP32 and split-BF16 MFMA against F
separate FP64 oracle gathers, one per field (the oracle has no GEMM).

Tolerances, per evaluation point and field, against the oracle's sum of
|terms| (cond):
  - FP32: as the single-field FP32 gather, u (300 + 4 (|x| + |z|) / r_min);
  - split-BF16: each operand is hi + lo with |lo| <= 2^-8 |x| and the dropped
    lo*lo term is <= 2^-16 |K C|; with FP32 accumulation the bound is
    2^-14 cond plus the FP32 term.
"""
import sys

import numpy as np
import pytest
import torch

from gpu_helpers import lib, to_np_aos

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _case(dim, N, K, F, seed):
    rng = np.random.default_rng(seed)
    th = rng.normal(0, 1, (N, dim))
    cy = th / np.linalg.norm(th, axis=1, keepdims=True)
    cn = cy.copy()
    A = rng.normal(0, 1, (N, F)) / N
    B = rng.normal(0, 1, (N, F)) / N
    r = 0.9 * rng.random(K) ** (1.0 / dim)
    d = rng.normal(0, 1, (K, dim))
    ex = d / np.linalg.norm(d, axis=1, keepdims=True) * r[:, None]
    return ex, cy, cn, A, B


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("F", [32, 64])
def test_gather_multi_matches_oracle(orc, dim, F):
    _bvc, pl = lib()
    say(f"gather_multi dim={dim} F={F}")
    ex, cy, cn, A, B = _case(dim, 300, 1000, F, dim * 7 + F)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to("cuda", torch.float32)
    cx_d, cn_d, ex_d = dev(cy.T), dev(cn.T), dev(ex.T)
    A_d, B_d = dev(A), dev(B)
    out = {}
    for prec in (_bvc.F32, _bvc.SPLIT_BF16):
        U = torch.empty(ex.shape[0], F, dtype=torch.float32, device="cuda")
        nb = _bvc.bvc_gather_multi_workspace_bytes(cy.shape[0], prec)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
        _bvc.bvc_gather_multi(dim, cy.shape[0], cx_d, cn_d, F, A_d, B_d, ex.shape[0], ex_d, U, prec, ws)
        torch.cuda.synchronize()
        out[prec] = U.double().cpu().numpy()
    # the oracle on the inputs as the device holds them
    cy_r, cn_r, ex_r = to_np_aos(cx_d), to_np_aos(cn_d), to_np_aos(ex_d)
    A_r, B_r = A_d.double().cpu().numpy(), B_d.double().cpu().numpy()
    rmin = np.min(np.linalg.norm(ex_r[:, None, :] - cy_r[None], axis=2), axis=1)
    fp32 = 2.0**-24 * (300 + 4 * (np.linalg.norm(ex_r, axis=1) + 1.01) / rmin)
    for f in range(F):
        uo, cond = orc.gather(dim, ex_r, cy_r, cn_r, A_r[:, f], B_r[:, f], with_grad=False, with_cond=True)
        assert np.all(np.abs(out[_bvc.F32][:, f] - uo) <= fp32 * cond), f
        assert np.all(np.abs(out[_bvc.SPLIT_BF16][:, f] - uo) <= (2.0**-14 + fp32) * cond), f
    err = np.abs(out[_bvc.SPLIT_BF16] - out[_bvc.F32]).max()
    say(f"  max |split-bf16 - fp32| = {err:.3e}")
