"""Thin ctypes binding of libbvc.so.

Each function has the name of the C entry point it calls and only marshals
arguments: torch tensors become device pointers, Python numbers become C
values, and a nonzero status becomes a BVCError carrying bvc_last_error().
Every computation runs in the library's kernels.  Importing this module fails
loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbvc.so")

F32 = 0
F64 = 1
SPLIT_BF16 = 2

ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED", -5: "ESTATE"}


class BVCError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


class bvc_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_coef", C.c_int32), ("coef", C.c_void_p),
                ("param", C.c_double * 8)]


class bvc_scene_info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_verts", C.c_int64), ("n_prims", C.c_int64),
                ("n_edges", C.c_int64), ("n_nodes", C.c_int64), ("depth", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("diagonal", C.c_double),
                ("boundary_measure", C.c_double), ("device_bytes", C.c_size_t),
                ("uploaded", C.c_int32)]


class bvc_walk_params(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_steps", C.c_int32), ("n_walks", C.c_int32),
                ("seed", C.c_uint64), ("batch", C.c_uint32), ("control_variate", C.c_int32),
                ("dtype", C.c_int32), ("blocks", C.c_int32), ("g", bvc_field), ("f", bvc_field),
                ("ev_begin", C.c_void_p), ("ev_end", C.c_void_p), ("sigma", C.c_double),
                ("open_center", C.c_double * 3), ("open_radius", C.c_double), ("side_read", C.c_int32),
                ("h", bvc_field), ("n_dev", C.c_void_p), ("order", C.c_void_p)]


class bvc_cache_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("dtype", C.c_int32), ("x", C.c_void_p), ("nrm", C.c_void_p),
                ("a", C.c_void_p), ("b", C.c_void_p), ("n_dev", C.c_void_p)]


class bvc_source_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("dtype", C.c_int32), ("y", C.c_void_p), ("s", C.c_void_p)]


class bvc_gather_params(C.Structure):
    _fields_ = [("accumulate", C.c_int32), ("near_tau", C.c_double), ("near_x", C.c_void_p),
                ("near_cx", C.c_void_p), ("near_cn", C.c_void_p), ("near_a", C.c_void_p),
                ("near_b", C.c_void_p), ("clamp_c", C.c_double), ("sigma", C.c_double), ("near_lead", C.c_int64)]


class bvc_clamp_params(C.Structure):
    _fields_ = [("l", C.c_double), ("sides", C.c_int32), ("c", C.c_double), ("n_rays", C.c_int32),
                ("max_hits", C.c_int32)]


class bvc_batch_item(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("walk", bvc_walk_params), ("n_cache", C.c_int64), ("x", C.c_void_p),
                ("nrm", C.c_void_p), ("R0", C.c_void_p), ("xbar", C.c_void_p), ("w", C.c_void_p),
                ("cx", C.c_void_p), ("cn", C.c_void_p), ("n_eval", C.c_int64), ("eval_x", C.c_void_p),
                ("u", C.c_void_p)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2302_11825_amd.build")

_L = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_P = C.POINTER

_SIGS = {
    "bvc_scene_create": [C.c_int32, _vp, C.c_int64, _vp, C.c_int64, _P(_vp)],
    "bvc_scene_get_info": [_vp, _P(bvc_scene_info)],
    "bvc_scene_upload": [_vp, _vp, C.c_size_t, _vp],
    "bvc_scene_destroy": [_vp],
    "bvc_scene_export_bvh": [_vp, _vp, _vp, _vp],
    "bvc_scene_export_slabs": [_vp, _vp],
    "bvc_cache_measure": [_vp, C.c_double, C.c_int32, _P(C.c_double)],
    "bvc_sample_cache": [_vp, C.c_int64, C.c_double, C.c_int32, C.c_uint64, C.c_uint32, _vp, _vp, _vp,
                         _vp, _vp, _vp, _vp],
    "bvc_sample_sources": [_vp, _P(bvc_field), C.c_int64, _P(C.c_double), _P(C.c_double), C.c_double,
                           C.c_uint64, C.c_uint32, _vp, _vp, _vp],
    "bvc_classify": [_vp, C.c_int64, _vp, C.c_double, _vp, _vp, _vp],
    "bvc_compact": [C.c_int64, _vp, C.c_int32, _vp, _vp, _P(C.c_int64), _vp],
    "bvc_take": [C.c_int32, C.c_int32, C.c_int64, _vp, C.c_int32, C.c_int64, _vp, C.c_int64, _vp, _vp],
    "bvc_compact_count": [C.c_int64, _vp, C.c_int32, _vp, _vp, _vp, _vp],
    "bvc_take_count": [C.c_int32, C.c_int32, C.c_int64, _vp, _vp, C.c_int32, C.c_int64, _vp, C.c_int64, _vp, _vp],
    "bvc_scatter": [C.c_int32, C.c_int64, _vp, C.c_int32, C.c_int64, _vp, C.c_int64, _vp, _vp],
    "bvc_spatial_order": [_vp, C.c_int32, C.c_int64, _vp, C.c_int64, _vp, _vp, _vp, C.c_size_t, _vp],
    "bvc_cache_walks": [_vp, _P(bvc_walk_params), C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                        _vp, _vp],
    "bvc_reduce_walks": [C.c_int64, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, _vp, _vp],
    "bvc_reduce_walks_count": [C.c_int64, _vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, _vp,
                               _vp],
    "bvc_pointwise_wos": [_vp, _P(bvc_walk_params), C.c_int64, _vp, _vp, _vp, _vp, C.c_size_t, _vp, _vp, _vp,
                          _vp],
    "bvc_pointwise_wos_noalloc": [_vp, _P(bvc_walk_params), C.c_int64, _vp, _vp, _vp, _vp, _vp],
    "bvc_gather_u": [C.c_int32, _P(bvc_cache_view), _P(bvc_source_view), C.c_int64, _vp, _vp,
                     _P(bvc_gather_params), _vp],
    "bvc_gather_grad": [C.c_int32, _P(bvc_cache_view), _P(bvc_source_view), C.c_int64, _vp, _vp, _vp,
                        _P(bvc_gather_params), _vp],
    "bvc_tune_gather": [C.c_int32, _P(bvc_cache_view), _P(bvc_source_view), C.c_int64, _vp, _vp, _vp,
                        _P(bvc_gather_params), C.c_int32, _P(C.c_int32), _vp],
    "bvc_tune_walks": [_vp, _P(bvc_walk_params), C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                       C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32), _vp],
    "bvc_tune_pointwise": [_vp, _P(bvc_walk_params), C.c_int64, _vp, _vp, _vp, _vp, C.c_size_t, _vp, _vp, _vp,
                           C.c_int32, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32), _vp],
    "bvc_gather_backward": [C.c_int32, _P(bvc_cache_view), _P(bvc_source_view), C.c_int64, _vp, _vp, _vp,
                            _vp, _vp, _vp, _vp],
    "bvc_basis_means": [_P(bvc_field), C.c_int32, C.c_int64, C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_int32,
                        _vp, _vp, _vp],
    "bvc_cache_backward": [C.c_int64, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "bvc_eval_fields": [C.c_int64, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, C.c_int32, _vp, _vp, _vp],
    "bvc_gather_multi": [C.c_int32, C.c_int64, _vp, _vp, C.c_int32, _vp, _vp, C.c_int64, _vp, _vp,
                         C.c_int32, _vp, C.c_size_t, _vp],
    "bvc_batch_plan": [_P(bvc_batch_item), C.c_int32, _vp, C.c_size_t, _vp, _P(_vp)],
    "bvc_batch_launch": [_vp, _vp],
    "bvc_batch_counters": [_vp, _P(_vp)],
    "bvc_batch_results": [_vp, _P(_vp), _P(_vp), _P(_vp), _P(_vp)],
    "bvc_batch_destroy": [_vp],
    "bvc_point_winding": [_vp, C.c_int64, _vp, _vp, _vp],
    "bvc_wost_walks": [_vp, _vp, _P(bvc_walk_params), C.c_int32, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                       _vp, C.c_size_t, _vp, _vp],
    "bvc_sample_roi": [_vp, _vp, C.c_int64, C.c_uint64, C.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "bvc_sample_mixed": [_vp, _vp, _vp, C.c_int64, C.c_double, C.c_double, C.c_uint64, C.c_uint32, _vp, _vp, _vp,
                         _vp, _vp, _vp, _vp],
    "bvc_classify_mixed": [_vp, _vp, C.c_int64, _vp, C.c_double, _vp, _vp, _vp],
    "bvc_clamp_correction": [_vp, _P(bvc_walk_params), _P(bvc_clamp_params), C.c_int64, _vp, _vp, _vp, _vp, _vp,
                             C.c_size_t, _vp, _vp],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_L, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int
_L.bvc_last_error.restype = C.c_char_p
_L.bvc_version.restype = C.c_char_p
_L.bvc_compact_scratch_ints.argtypes = [C.c_int64]
_L.bvc_compact_scratch_ints.restype = C.c_int64
_L.bvc_cache_backward_scratch_doubles.argtypes = [C.c_int64, C.c_int32]
_L.bvc_cache_backward_scratch_doubles.restype = C.c_int64
_L.bvc_pointwise_workspace_bytes.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32]
_L.bvc_pointwise_workspace_bytes.restype = C.c_size_t
_L.bvc_gather_multi_workspace_bytes.argtypes = [C.c_int64, C.c_int32]
_L.bvc_gather_multi_workspace_bytes.restype = C.c_size_t
_L.bvc_batch_workspace_bytes.argtypes = [_P(bvc_batch_item), C.c_int32]
_L.bvc_batch_workspace_bytes.restype = C.c_size_t
_L.bvc_wost_workspace_bytes.argtypes = [_vp]
_L.bvc_wost_workspace_bytes.restype = C.c_size_t
_L.bvc_clamp_radius.argtypes = [C.c_int32, C.c_double]
_L.bvc_clamp_radius.restype = C.c_double
_L.bvc_clamp_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32]
_L.bvc_clamp_workspace_bytes.restype = C.c_size_t
_L.bvc_pointwise_static_bytes.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32]
_L.bvc_pointwise_static_bytes.restype = C.c_size_t
_L.bvc_spatial_order_workspace_bytes.argtypes = []
_L.bvc_spatial_order_workspace_bytes.restype = C.c_size_t

# size of the library's static scratch of bvc_pointwise_wos_noalloc
POINTWISE_STATIC_BYTES = 32 << 20

EXPORTED = sorted(list(_SIGS) + ["bvc_last_error", "bvc_version", "bvc_compact_scratch_ints",
                                 "bvc_cache_backward_scratch_doubles", "bvc_pointwise_workspace_bytes",
                                 "bvc_gather_multi_workspace_bytes", "bvc_batch_workspace_bytes",
                                 "bvc_clamp_radius", "bvc_clamp_workspace_bytes", "bvc_wost_workspace_bytes",
                                 "bvc_pointwise_static_bytes", "bvc_spatial_order_workspace_bytes"])


def _check(rc, name):
    if rc != 0:
        raise BVCError(rc, name, _L.bvc_last_error().decode())


def ptr(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def dtype_code(t: torch.dtype) -> int:
    if t == torch.float32:
        return F32
    if t == torch.float64:
        return F64
    raise ValueError(f"unsupported dtype {t}")


def make_field(kind, coef_dev, param) -> bvc_field:
    f = bvc_field()
    f.kind = int(kind)
    f.n_coef = 0 if coef_dev is None else int(coef_dev.numel())
    f.coef = None if coef_dev is None or coef_dev.numel() == 0 else coef_dev.data_ptr()
    for i in range(8):
        f.param[i] = float(param[i]) if i < len(param) else 0.0
    return f


def bvc_version() -> str:
    return _L.bvc_version().decode()


def bvc_last_error() -> str:
    return _L.bvc_last_error().decode()


def bvc_compact_scratch_ints(n: int) -> int:
    return int(_L.bvc_compact_scratch_ints(n))


def bvc_cache_backward_scratch_doubles(n_cache: int, nb: int) -> int:
    return int(_L.bvc_cache_backward_scratch_doubles(n_cache, nb))


def bvc_scene_create(dim, verts, prims):
    """verts: host float64 (nv, dim); prims: host int32 (np, dim)."""
    import numpy as np

    v = np.ascontiguousarray(verts, dtype=np.float64)
    p = np.ascontiguousarray(prims, dtype=np.int32)
    h = C.c_void_p()
    _check(_L.bvc_scene_create(dim, v.ctypes.data, v.shape[0], p.ctypes.data, p.shape[0], C.byref(h)),
           "bvc_scene_create")
    return h


def bvc_scene_get_info(scene) -> bvc_scene_info:
    info = bvc_scene_info()
    _check(_L.bvc_scene_get_info(scene, C.byref(info)), "bvc_scene_get_info")
    return info


def bvc_scene_export_bvh(scene):
    """Host copy of the BVH topology: (child int32 [n_nodes, 2], boxes float64
    [n_nodes, 4*dim], order int32 [n_prims])."""
    import numpy as np

    info = bvc_scene_get_info(scene)
    child = np.empty((info.n_nodes, 2), dtype=np.int32)
    boxes = np.empty((info.n_nodes, 4 * info.dim), dtype=np.float64)
    order = np.empty(info.n_prims, dtype=np.int32)
    _check(_L.bvc_scene_export_bvh(scene, child.ctypes.data, boxes.ctypes.data, order.ctypes.data),
           "bvc_scene_export_bvh")
    return child, boxes, order


def bvc_scene_export_slabs(scene):
    """Host copy of the 3D slab bounds, float64 [n_nodes, 12]."""
    import numpy as np

    info = bvc_scene_get_info(scene)
    slabs = np.empty((info.n_nodes, 12), dtype=np.float64)
    _check(_L.bvc_scene_export_slabs(scene, slabs.ctypes.data), "bvc_scene_export_slabs")
    return slabs


def bvc_scene_upload(scene, buf, stream=None):
    _check(_L.bvc_scene_upload(scene, ptr(buf), buf.numel() * buf.element_size(), stream_ptr(stream)),
           "bvc_scene_upload")


def bvc_scene_destroy(scene):
    _check(_L.bvc_scene_destroy(scene), "bvc_scene_destroy")


def bvc_cache_measure(scene, l, sides) -> float:
    m = C.c_double()
    _check(_L.bvc_cache_measure(scene, l, sides, C.byref(m)), "bvc_cache_measure")
    return m.value


def bvc_sample_roi(dom, roi, n, seed, batch, x, nrm, w, xbar, R0, accept, stream=None):
    _check(_L.bvc_sample_roi(dom, roi, n, seed, batch, ptr(x), ptr(nrm), ptr(w), ptr(xbar), ptr(R0), ptr(accept),
                             stream_ptr(stream)), "bvc_sample_roi")


def bvc_sample_mixed(full, dir_scene, neu, n, l, seed, batch, x, nrm, w, xbar, R0, kind, stream=None,
                     junction_drop=0.0):
    _check(_L.bvc_sample_mixed(full, dir_scene, neu, n, l, float(junction_drop), seed, batch, ptr(x), ptr(nrm), ptr(w),
                               ptr(xbar), ptr(R0), ptr(kind), stream_ptr(stream)), "bvc_sample_mixed")


def bvc_classify_mixed(full, dir_scene, n, x, l, cls, dist=None, stream=None):
    _check(_L.bvc_classify_mixed(full, dir_scene, n, ptr(x), l, ptr(cls), ptr(dist), stream_ptr(stream)),
           "bvc_classify_mixed")


def bvc_sample_cache(scene, n, l, sides, seed, batch, x, nrm, w, xbar, R0, accept, stream=None):
    _check(_L.bvc_sample_cache(scene, n, l, sides, seed, batch, ptr(x), ptr(nrm), ptr(w), ptr(xbar), ptr(R0),
                               ptr(accept), stream_ptr(stream)), "bvc_sample_cache")


def bvc_sample_sources(scene, f: bvc_field, m, lo, hi, l, seed, batch, y, s, stream=None):
    lo_c = (C.c_double * 3)(*[float(v) for v in lo])
    hi_c = (C.c_double * 3)(*[float(v) for v in hi])
    _check(_L.bvc_sample_sources(scene, C.byref(f), m, lo_c, hi_c, l, seed, batch, ptr(y), ptr(s),
                                 stream_ptr(stream)), "bvc_sample_sources")


def bvc_classify(scene, n, x, l, cls, dist=None, stream=None):
    _check(_L.bvc_classify(scene, n, ptr(x), l, ptr(cls), ptr(dist), stream_ptr(stream)), "bvc_classify")


def bvc_compact(n, flags, want, idx, scratch, stream=None) -> int:
    cnt = C.c_int64()
    _check(_L.bvc_compact(n, ptr(flags), want, ptr(idx), ptr(scratch), C.byref(cnt), stream_ptr(stream)),
           "bvc_compact")
    return cnt.value


def bvc_compact_count(n, flags, want, idx, scratch, count, stream=None):
    """Compaction with the count left on the device (int64 tensor `count`)."""
    _check(_L.bvc_compact_count(n, ptr(flags), want, ptr(idx), ptr(scratch), ptr(count), stream_ptr(stream)),
           "bvc_compact_count")


def bvc_take_count(dtype_in, dtype_out, n_cap, count, idx, rows, ld_in, src, ld_out, out, stream=None):
    _check(_L.bvc_take_count(dtype_in, dtype_out, n_cap, ptr(count), ptr(idx), rows, ld_in, ptr(src), ld_out,
                             ptr(out), stream_ptr(stream)), "bvc_take_count")


def bvc_take(dtype_in, dtype_out, n_idx, idx, rows, ld_in, src, ld_out, out, stream=None):
    _check(_L.bvc_take(dtype_in, dtype_out, n_idx, ptr(idx), rows, ld_in, ptr(src), ld_out, ptr(out),
                       stream_ptr(stream)), "bvc_take")


def bvc_scatter(dtype, n_idx, idx, rows, ld_in, src, ld_out, out, stream=None):
    _check(_L.bvc_scatter(dtype, n_idx, ptr(idx), rows, ld_in, ptr(src), ld_out, ptr(out), stream_ptr(stream)),
           "bvc_scatter")


def bvc_spatial_order_workspace_bytes():
    return int(_L.bvc_spatial_order_workspace_bytes())


def bvc_spatial_order(scene, n, x, order, work, n_dev=None, stream=None):
    """x: [dim][ld] FP32 or FP64 device points; order: int32 [n] device."""
    _check(_L.bvc_spatial_order(scene, dtype_code(x.dtype), n, ptr(x), x.shape[1] if x.dim() == 2 else 0,
                                ptr(n_dev), ptr(order), ptr(work), work.numel() * work.element_size(),
                                stream_ptr(stream)), "bvc_spatial_order")


def bvc_cache_walks(scene, params: bvc_walk_params, n_cache, x, nrm, R0, xbar, U, D, rec_exit=None,
                    rec_w1=None, rec_steps=None, counters=None, stream=None):
    _check(_L.bvc_cache_walks(scene, C.byref(params), n_cache, ptr(x), ptr(nrm), ptr(R0), ptr(xbar), ptr(U),
                              ptr(D), ptr(rec_exit), ptr(rec_w1), ptr(rec_steps), ptr(counters),
                              stream_ptr(stream)), "bvc_cache_walks")


def bvc_reduce_walks(n_cache, W, dtype_in, U, D, w, uhat, dudn, dtype_out, a, b, stream=None):
    _check(_L.bvc_reduce_walks(n_cache, W, dtype_in, ptr(U), ptr(D), ptr(w), ptr(uhat), ptr(dudn), dtype_out,
                               ptr(a), ptr(b), stream_ptr(stream)), "bvc_reduce_walks")


def bvc_reduce_walks_count(n_cap, count, W, dtype_in, U, D, w, uhat, dudn, dtype_out, a, b, stream=None):
    _check(_L.bvc_reduce_walks_count(n_cap, ptr(count), W, dtype_in, ptr(U), ptr(D), ptr(w), ptr(uhat), ptr(dudn),
                                     dtype_out, ptr(a), ptr(b), stream_ptr(stream)), "bvc_reduce_walks_count")


def bvc_tune_pointwise(scene, params: bvc_walk_params, n, x, U_walk, G_walk, work, u, grad, counters, reps=2,
                       stream=None):
    """Returns (blocks per compute unit, open lanes, slab bounds on) the library
    keeps for this class of pointwise walks."""
    bpc, lanes, slabs = C.c_int32(), C.c_int32(), C.c_int32()
    nbytes = work.numel() * work.element_size() if work is not None else 0
    _check(_L.bvc_tune_pointwise(scene, C.byref(params), n, ptr(x), ptr(U_walk), ptr(G_walk), ptr(work), nbytes,
                                 ptr(u), ptr(grad), ptr(counters), reps, C.byref(bpc), C.byref(lanes),
                                 C.byref(slabs), stream_ptr(stream)), "bvc_tune_pointwise")
    return bpc.value, lanes.value, slabs.value


def bvc_pointwise_workspace_bytes(dim, n, W, dtype, with_grad) -> int:
    return int(_L.bvc_pointwise_workspace_bytes(dim, n, W, dtype, int(bool(with_grad))))


def bvc_pointwise_wos(scene, params: bvc_walk_params, n, x, U_walk, G_walk, work, u, grad, counters,
                      stream=None):
    nbytes = 0 if work is None else work.numel() * work.element_size()
    _check(_L.bvc_pointwise_wos(scene, C.byref(params), n, ptr(x), ptr(U_walk), ptr(G_walk), ptr(work), nbytes,
                                ptr(u), ptr(grad), ptr(counters), stream_ptr(stream)), "bvc_pointwise_wos")


def bvc_pointwise_static_bytes(dim, n, W, dtype, with_grad) -> int:
    return int(_L.bvc_pointwise_static_bytes(dim, n, W, dtype, int(bool(with_grad))))


def bvc_pointwise_wos_noalloc(scene, params: bvc_walk_params, n, x, u, grad, counters, stream=None):
    _check(_L.bvc_pointwise_wos_noalloc(scene, C.byref(params), n, ptr(x), ptr(u), ptr(grad), ptr(counters),
                                        stream_ptr(stream)), "bvc_pointwise_wos_noalloc")


def _views(cache, sources):
    cv = bvc_cache_view()
    cv.n, cv.dtype = cache["n"], cache["dtype"]
    cv.x, cv.nrm, cv.a, cv.b = (t.data_ptr() if t is not None else None
                                for t in (cache["x"], cache["nrm"], cache["a"], cache["b"]))
    n_dev = cache.get("n_dev")
    cv.n_dev = n_dev.data_ptr() if n_dev is not None else None
    sv = None
    if sources is not None:
        sv = bvc_source_view()
        sv.n, sv.dtype = sources["n"], sources["dtype"]
        sv.y = sources["y"].data_ptr() if sources["n"] else None
        sv.s = sources["s"].data_ptr() if sources["n"] else None
    return cv, sv


def _gparams(accumulate, near, clamp=0.0, sigma=0.0):
    """near: None, or dict(tau, x, cx, cn, a, b[, lead]) with FP64 device
    tensors (evaluation points [dim][n_eval], cache points and normals
    [dim][n], a, b); lead: the number of leading evaluation points that can
    need the near field (0 = all).
    clamp: bound c of dG/dn in the potential (Eq. 9), 0 = off."""
    gp = bvc_gather_params()
    gp.accumulate = accumulate
    gp.clamp_c = float(clamp)
    gp.sigma = float(sigma)
    if near is not None:
        gp.near_tau = float(near["tau"])
        gp.near_x, gp.near_cx, gp.near_cn, gp.near_a, gp.near_b = (
            ptr(near[k]) for k in ("x", "cx", "cn", "a", "b"))
        gp.near_lead = int(near.get("lead", 0))
    return gp


def bvc_gather_u(dim, cache, sources, n_eval, eval_x, u, accumulate=0, stream=None, near=None, clamp=0.0,
                 sigma=0.0):
    cv, sv = _views(cache, sources)
    gp = _gparams(accumulate, near, clamp, sigma)
    _check(_L.bvc_gather_u(dim, C.byref(cv), C.byref(sv) if sv is not None else None, n_eval, ptr(eval_x),
                           ptr(u), C.byref(gp), stream_ptr(stream)), "bvc_gather_u")


def bvc_gather_grad(dim, cache, sources, n_eval, eval_x, u, grad, accumulate=0, stream=None, near=None,
                    clamp=0.0, sigma=0.0):
    cv, sv = _views(cache, sources)
    gp = _gparams(accumulate, near, clamp, sigma)
    _check(_L.bvc_gather_grad(dim, C.byref(cv), C.byref(sv) if sv is not None else None, n_eval, ptr(eval_x),
                              ptr(u), ptr(grad), C.byref(gp), stream_ptr(stream)), "bvc_gather_grad")


def bvc_tune_gather(dim, cache, sources, n_eval, eval_x, u, grad=None, reps=3, stream=None, near=None):
    """Returns the points-per-thread the library keeps for this gather class."""
    cv, sv = _views(cache, sources)
    gp = _gparams(0, near)
    out = C.c_int32()
    _check(_L.bvc_tune_gather(dim, C.byref(cv), C.byref(sv) if sv is not None else None, n_eval, ptr(eval_x),
                              ptr(u), ptr(grad), C.byref(gp), reps, C.byref(out), stream_ptr(stream)),
           "bvc_tune_gather")
    return out.value


def bvc_tune_walks(scene, params: bvc_walk_params, n_cache, x, nrm, R0, xbar, U, D, rec_exit, rec_w1, counters,
                   reps=2, stream=None):
    """Returns (blocks per compute unit, open lanes, slab bounds on) the library
    keeps for this walk class."""
    bpc, lanes, slabs = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_L.bvc_tune_walks(scene, C.byref(params), n_cache, ptr(x), ptr(nrm), ptr(R0), ptr(xbar), ptr(U), ptr(D),
                             ptr(rec_exit), ptr(rec_w1), ptr(counters), reps, C.byref(bpc), C.byref(lanes),
                             C.byref(slabs), stream_ptr(stream)), "bvc_tune_walks")
    return bpc.value, lanes.value, slabs.value


def bvc_gather_backward(dim, cache, sources, n_eval, eval_x, dL_du, dL_da, dL_db, dL_ds=None, dL_dx=None,
                        stream=None):
    cv, sv = _views(cache, sources)
    _check(_L.bvc_gather_backward(dim, C.byref(cv), C.byref(sv) if sv is not None else None, n_eval,
                                  ptr(eval_x), ptr(dL_du), ptr(dL_da), ptr(dL_db), ptr(dL_ds), ptr(dL_dx),
                                  stream_ptr(stream)), "bvc_gather_backward")


def bvc_basis_means(basis: bvc_field, dim, n_cache, W, dtype, rec_exit, rec_w1, xbar, cv, E, F, stream=None):
    _check(_L.bvc_basis_means(C.byref(basis), dim, n_cache, W, dtype, ptr(rec_exit), ptr(rec_w1), ptr(xbar), cv,
                              ptr(E), ptr(F), stream_ptr(stream)), "bvc_basis_means")


def bvc_cache_backward(n_cache, nb, E, F, w, dL_da, dL_db, scratch, dL_dtheta, stream=None):
    _check(_L.bvc_cache_backward(n_cache, nb, ptr(E), ptr(F), ptr(w), ptr(dL_da), ptr(dL_db), ptr(scratch),
                                 ptr(dL_dtheta), stream_ptr(stream)), "bvc_cache_backward")


def bvc_eval_fields(n_cache, nb, n_fields, E, F, w, coef, dtype_out, A, B, stream=None):
    _check(_L.bvc_eval_fields(n_cache, nb, n_fields, ptr(E), ptr(F), ptr(w), ptr(coef), dtype_out, ptr(A),
                              ptr(B), stream_ptr(stream)), "bvc_eval_fields")


def bvc_batch_workspace_bytes(items) -> int:
    arr = (bvc_batch_item * len(items))(*items)
    return int(_L.bvc_batch_workspace_bytes(arr, len(items)))


def bvc_batch_plan(items, workspace, stream=None):
    arr = (bvc_batch_item * len(items))(*items)
    h = C.c_void_p()
    _check(_L.bvc_batch_plan(arr, len(items), ptr(workspace), workspace.numel() * workspace.element_size(),
                             stream_ptr(stream), C.byref(h)), "bvc_batch_plan")
    return h


def bvc_batch_launch(batch, stream=None):
    _check(_L.bvc_batch_launch(batch, stream_ptr(stream)), "bvc_batch_launch")


def bvc_batch_counters(batch) -> int:
    p = C.c_void_p()
    _check(_L.bvc_batch_counters(batch, C.byref(p)), "bvc_batch_counters")
    return p.value


def bvc_batch_results(batch):
    """Device addresses (U, D, a, b) of the batch's per-walk samples and cache values."""
    ps = [C.c_void_p() for _ in range(4)]
    _check(_L.bvc_batch_results(batch, *(C.byref(p) for p in ps)), "bvc_batch_results")
    return tuple(p.value for p in ps)


def bvc_batch_destroy(batch):
    _check(_L.bvc_batch_destroy(batch), "bvc_batch_destroy")


def bvc_gather_multi_workspace_bytes(n_cache, precision) -> int:
    return int(_L.bvc_gather_multi_workspace_bytes(n_cache, precision))


def bvc_gather_multi(dim, n_cache, cx, cn, n_fields, A, B, n_eval, eval_x, U, precision, workspace=None,
                     stream=None):
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_L.bvc_gather_multi(dim, n_cache, ptr(cx), ptr(cn), n_fields, ptr(A), ptr(B), n_eval, ptr(eval_x),
                               ptr(U), precision, ptr(workspace), nbytes, stream_ptr(stream)), "bvc_gather_multi")


def bvc_clamp_radius(dim, c):
    return _L.bvc_clamp_radius(dim, float(c))


def bvc_point_winding(scene, n, x, wind, stream=None):
    _check(_L.bvc_point_winding(scene, n, ptr(x), ptr(wind), stream_ptr(stream)), "bvc_point_winding")


def bvc_clamp_workspace_bytes(dim, dtype, n, n_rays, max_hits):
    return _L.bvc_clamp_workspace_bytes(dim, dtype, n, n_rays, max_hits)


def clamp_params(l, sides, c, n_rays, max_hits):
    cp = bvc_clamp_params()
    cp.l, cp.sides, cp.c, cp.n_rays, cp.max_hits = float(l), int(sides), float(c), int(n_rays), int(max_hits)
    return cp


def bvc_clamp_correction(scene, params: bvc_walk_params, cp: bvc_clamp_params, n, x, wind, out_index, u, work,
                         counters, stream=None):
    nbytes = 0 if work is None else work.numel() * work.element_size()
    _check(_L.bvc_clamp_correction(scene, C.byref(params), C.byref(cp), n, ptr(x), ptr(wind), ptr(out_index), ptr(u),
                                   ptr(work), nbytes, ptr(counters), stream_ptr(stream)), "bvc_clamp_correction")


def bvc_wost_workspace_bytes(neu):
    return _L.bvc_wost_workspace_bytes(neu)


def bvc_wost_walks(dir_scene, neu_scene, params: bvc_walk_params, mode, n, x, nrm, R0, xbar, U, D, steps, work,
                   counters, stream=None):
    nbytes = 0 if work is None else work.numel() * work.element_size()
    _check(_L.bvc_wost_walks(dir_scene, neu_scene, C.byref(params), mode, n, ptr(x), ptr(nrm), ptr(R0), ptr(xbar),
                             ptr(U), ptr(D), ptr(steps), ptr(work), nbytes, ptr(counters), stream_ptr(stream)),
           "bvc_wost_walks")
