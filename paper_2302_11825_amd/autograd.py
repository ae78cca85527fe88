"""Differentiation through the cache and the gather with hand-written adjoints.

For fixed walks every estimator of the method is linear in the boundary data:
with the walks' exit records, u-hat = E theta and du/dn-hat = F theta for
g = sum_m theta_m phi_m (E, F from bvc_basis_means), so the cache values are
a = w * (E theta), b = w * (F theta).  The gather (Eqs. 3-6) is linear in
(a, b, s) and smooth in the evaluation positions.

  CacheFunction:  theta -> (a, b)          backward: bvc_cache_backward
  GatherFunction: (a, b, s, x) -> u        backward: bvc_gather_backward
                                            (dL/dx = dL/du * grad u, Eq. 5-6)

The walks are never re-run: the exit records are the checkpoint.  Every
forward and backward step is a library kernel; torch only allocates.
"""
from __future__ import annotations

import torch

from . import _bvc as B


def _code(t):
    return B.dtype_code(t.dtype)


class CacheFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, E, F, w, dtype=torch.float64):
        n, nb = E.shape
        dev = E.device
        coef = theta.detach().reshape(1, nb)
        if coef.dtype != torch.float64 or not coef.is_contiguous():
            c64 = torch.empty(1, nb, dtype=torch.float64, device=dev)
            B.bvc_take(_code(coef), B.F64, nb, None, 1, nb, coef.contiguous(), nb, c64)
            coef = c64
        a = torch.empty(n, 1, dtype=dtype, device=dev)
        b = torch.empty(n, 1, dtype=dtype, device=dev)
        B.bvc_eval_fields(n, nb, 1, E, F, w, coef, B.dtype_code(dtype), a, b)
        ctx.save_for_backward(E, F, w)
        ctx.theta_dtype = theta.dtype
        return a.view(n), b.view(n)

    @staticmethod
    def backward(ctx, ga, gb):
        E, F, w = ctx.saved_tensors
        n, nb = E.shape
        dev = E.device

        def as64(g):
            out = torch.zeros(n, dtype=torch.float64, device=dev)
            if g is not None:
                g = g.contiguous()
                B.bvc_take(_code(g), B.F64, n, None, 1, n, g, n, out)
            return out

        scratch = torch.empty(B.bvc_cache_backward_scratch_doubles(n, nb), dtype=torch.float64, device=dev)
        out = torch.empty(nb, dtype=torch.float64, device=dev)
        B.bvc_cache_backward(n, nb, E, F, w, as64(ga), as64(gb), scratch, out)
        if ctx.theta_dtype != torch.float64:
            o = torch.empty(nb, dtype=ctx.theta_dtype, device=dev)
            B.bvc_take(B.F64, B.dtype_code(ctx.theta_dtype), nb, None, 1, nb, out, nb, o)
            out = o
        return out, None, None, None, None


class GatherFunction(torch.autograd.Function):
    """u = gather(a, b, s; x) with cache points cx, normals cn ([dim][N]),
    sources sy ([dim][M], optional) and evaluation points x ([dim][K])."""

    @staticmethod
    def forward(ctx, a, b, s, x, cx, cn, sy):
        dim, K = x.shape
        dt = a.dtype
        code = B.dtype_code(dt)
        cache = dict(n=cx.shape[1], dtype=code, x=cx, nrm=cn, a=a.contiguous(), b=b.contiguous())
        src = dict(n=sy.shape[1], dtype=code, y=sy, s=s.contiguous()) if s is not None else None
        u = torch.empty(K, dtype=dt, device=a.device)
        B.bvc_gather_u(dim, cache, src, K, x.contiguous(), u)
        ctx.save_for_backward(a, b, s if s is not None else a.new_empty(0), x, cx, cn,
                              sy if sy is not None else a.new_empty(0, 0))
        ctx.has_src = s is not None
        return u

    @staticmethod
    def backward(ctx, gu):
        a, b, s, x, cx, cn, sy = ctx.saved_tensors
        dim, K = x.shape
        code = B.dtype_code(a.dtype)
        cache = dict(n=cx.shape[1], dtype=code, x=cx, nrm=cn, a=a, b=b)
        src = dict(n=sy.shape[1], dtype=code, y=sy, s=s) if ctx.has_src else None
        gu = gu.contiguous()
        da = torch.empty_like(a) if ctx.needs_input_grad[0] else None
        db = torch.empty_like(b) if ctx.needs_input_grad[1] else None
        ds = torch.empty_like(s) if (ctx.has_src and ctx.needs_input_grad[2]) else None
        dx = torch.empty_like(x) if ctx.needs_input_grad[3] else None
        B.bvc_gather_backward(dim, cache, src, K, x, gu, da, db, ds, dx)
        return da, db, ds, dx, None, None, None


def gather(a, b, x, cx, cn, s=None, sy=None):
    return GatherFunction.apply(a, b, s, x, cx, cn, sy)


def cache_values(theta, E, F, w, dtype=torch.float64):
    return CacheFunction.apply(theta, E, F, w, dtype)
