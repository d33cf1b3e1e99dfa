"""Python binding of the C ABI in include/gs.h (argument marshalling only).

Every function here takes torch tensors that live on a ROCm device, allocates
the outputs and the workspace with torch, and calls the entry point of the
same name in libgsbh.so on torch's current stream.  All arithmetic runs in the
library's HIP kernels; if the library is missing this module raises instead
of computing anything itself.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# GSBH_LIB selects another build of the library (the host-sanitized build of
# the sanitizer checks); by default the in-tree libgsbh.so.
LIB_PATH = os.environ.get("GSBH_LIB") or os.path.join(_PKG, "libgsbh.so")

GS_EXACT, GS_BH = 0, 1
GS_OP_RHS, GS_OP_SHOOT, GS_OP_ADJOINT, GS_OP_FIELD = 0, 1, 2, 3
GS_FLAG_F64 = 1
GS_FLAG_GRAPH = 4
STATUS = {0: "GS_OK", -1: "GS_ERR_INVALID", -2: "GS_ERR_WORKSPACE", -3: "GS_ERR_HIP",
          -4: "GS_ERR_NONFINITE", -5: "GS_ERR_UNSUPPORTED", -6: "GS_ERR_OVERFLOW"}


class GsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("cutoff_sigmas", ctypes.c_double),
                ("theta", ctypes.c_double), ("leaf_cap", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("exact_items", ctypes.c_int32)]


def params(sigma, nt=40, theta=0.5, cutoff_sigmas=3.0, leaf_cap=1, flags=0,
           exact_items=0) -> Params:
    return Params(float(sigma), float(cutoff_sigmas), float(theta), int(leaf_cap),
                  int(nt), int(flags), int(exact_items))


_lib = None
_vp, _i64, _i32, _sz, _dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_size_t, ctypes.c_double)
_PP = ctypes.POINTER(Params)

# name -> (restype, argtypes); the order follows include/gs.h
_SIGS = {
    "gs_version": (ctypes.c_char_p, []),
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_params_default": (None, [_PP]),
    "gs_workspace_bytes": (_sz, [_i64, _PP, _i32, _i32]),
    "gs_rhs_exact": (ctypes.c_int, [_vp, _vp, _i64, _PP, _vp, _vp, _vp, _sz, _vp]),
    "gs_rhs_exact_f64": (ctypes.c_int, [_vp, _vp, _i64, _PP, _vp, _vp, _vp, _sz, _vp]),
    "gs_rhs_bh": (ctypes.c_int, [_vp, _vp, _i64, _PP, _vp, _vp, _vp, _sz, _vp]),
    "gs_shoot": (ctypes.c_int, [_vp, _vp, _i64, _PP, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gs_shoot_f64": (ctypes.c_int, [_vp, _vp, _i64, _PP, _vp, _vp, _vp, _vp, _sz, _vp]),
    "gs_shoot_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _i64, _PP, _i32, _dbl, _i32, _vp,
                                        _vp, _vp, _sz, _vp]),
    "gs_adjoint_workspace_bytes": (_sz, [_i64, _PP, _i32, _i32]),
    "gs_field_workspace_bytes": (_sz, [_i64, _i64, _PP]),
    "gs_field": (ctypes.c_int, [_vp, _i64, _vp, _vp, _i64, _PP, _vp, _vp, _sz, _vp]),
    "gs_batch_workspace_bytes": (_sz, [_vp, _i32, _PP, _i32, _i32]),
    "gs_rhs_batch": (ctypes.c_int, [_vp, _vp, _vp, _i32, _PP, _i32, _vp, _vp, _vp, _sz, _vp]),
    "gs_shoot_batch": (ctypes.c_int, [_vp, _vp, _vp, _i32, _PP, _i32, _vp, _vp, _vp, _vp, _sz,
                                      _vp]),
    "gs_adjoint_batch_workspace_bytes": (_sz, [_vp, _i32, _PP, _i32, _i32]),
    "gs_shoot_adjoint_batch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _PP, _i32, _dbl, _i32,
                                              _vp, _vp, _vp, _sz, _vp]),
    "gs_autotune_leaf_cap": (ctypes.c_int, [_vp, _vp, _vp, _i32, _PP, _vp, _vp, _vp, _sz,
                                            _vp, ctypes.POINTER(ctypes.c_double)]),
    "gs_autotune_exact": (ctypes.c_int, [_vp, _vp, _vp, _i32, _PP, _vp, _vp, _vp, _sz, _vp,
                                         ctypes.POINTER(ctypes.c_double)]),
    "gs_tree_export": (ctypes.c_int, [_vp, _vp, _i64, _PP, _vp, _sz, _vp, _i64,
                                      ctypes.POINTER(ctypes.c_int64), _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp]),
    "gs_rhs_exact_static": (ctypes.c_int, [_vp, _vp, _i64, _PP, _vp, _vp, _vp]),
    "gs_get_status": (ctypes.c_int, [_vp, _vp]),
    "gs_bh_counters": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "gs_kernel_timing": (ctypes.c_int, [_i32]),
    "gs_kernel_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_double)]),
}
EXPORTS = tuple(_SIGS)


def lib():
    """Load libgsbh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1907_04834_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise GsError(status, lib().gs_last_error().decode())


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else None


def _pts(x, dtype, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a ROCm device tensor")
    if x.dtype != dtype or x.dim() != 2 or x.shape[1] != 3 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous ({dtype}) tensor of shape (n, 3)")
    return x


def _workspace(n, prm, method, op, dev):
    nbytes = lib().gs_workspace_bytes(n, ctypes.byref(prm), method, op)
    if nbytes == 0:
        raise GsError(-1, "invalid arguments for gs_workspace_bytes")
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)


def gs_version() -> str:
    return lib().gs_version().decode()


def gs_workspace_bytes(n, prm: Params, method=GS_EXACT, op=GS_OP_RHS) -> int:
    return int(lib().gs_workspace_bytes(n, ctypes.byref(prm), method, op))


def gs_rhs_exact(q, p, prm: Params, ws=None):
    """(dq, dp) = (v, a) of the exact right-hand side; float32 (n, 3)."""
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    n = q.shape[0]
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    if ws is None:
        ws = _workspace(n, prm, GS_EXACT, GS_OP_RHS, q.device)
    _check(lib().gs_rhs_exact(_ptr(q), _ptr(p), n, ctypes.byref(prm), _ptr(dq), _ptr(dp),
                              _ptr(ws), ws.numel(), _stream(q.device)))
    return dq, dp


def gs_rhs_exact_static(q, p, prm: Params, out=None):
    """gs_rhs_exact with the library's static device workspace (no workspace
    argument, no device allocation by the library; n <= GS_STATIC_MAX_N).
    `out` = (dq, dp) lets a caller that cannot allocate pass its own outputs."""
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    n = q.shape[0]
    if out is None:
        dq, dp = torch.empty_like(q), torch.empty_like(q)
    else:
        dq, dp = _pts(out[0], torch.float32, "dq"), _pts(out[1], torch.float32, "dp")
        if dq.shape != q.shape or dp.shape != q.shape:
            raise ValueError("dq / dp must have the shape of q")
    _check(lib().gs_rhs_exact_static(_ptr(q), _ptr(p), n, ctypes.byref(prm), _ptr(dq),
                                     _ptr(dp), _stream(q.device)))
    return dq, dp


GS_STATIC_SCRATCH_BYTES = 64 << 20
GS_STATIC_MAX_N = 500000


def gs_rhs_exact_f64(q, p, prm: Params):
    _pts(q, torch.float64, "q")
    _pts(p, torch.float64, "p")
    n = q.shape[0]
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    pr = Params.from_buffer_copy(prm)
    pr.flags |= GS_FLAG_F64
    ws = _workspace(n, pr, GS_EXACT, GS_OP_RHS, q.device)
    _check(lib().gs_rhs_exact_f64(_ptr(q), _ptr(p), n, ctypes.byref(prm), _ptr(dq),
                                  _ptr(dp), _ptr(ws), ws.numel(), _stream(q.device)))
    return dq, dp


def gs_rhs_bh(q, p, prm: Params, ws=None, return_ws=False):
    """(dq, dp) of the Barnes-Hut right-hand side; float32 (n, 3)."""
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    n = q.shape[0]
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    if ws is None:
        ws = _workspace(n, prm, GS_BH, GS_OP_RHS, q.device)
    _check(lib().gs_rhs_bh(_ptr(q), _ptr(p), n, ctypes.byref(prm), _ptr(dq), _ptr(dp),
                           _ptr(ws), ws.numel(), _stream(q.device)))
    return (dq, dp, ws) if return_ws else (dq, dp)


def _outputs(out, q0, hshape, with_energy):
    """(q1, p1, H): the caller's buffers `out`, checked, or new ones.  Passing
    the same buffers again lets a GS_FLAG_GRAPH call replay its graph."""
    if out is None:
        H = torch.zeros(hshape, dtype=torch.float64, device=q0.device) if with_energy else None
        return torch.empty_like(q0), torch.empty_like(q0), H
    q1, p1, H = out
    _pts(q1, torch.float32, "q1")
    _pts(p1, torch.float32, "p1")
    if q1.shape != q0.shape or p1.shape != q0.shape:
        raise ValueError("q1 / p1 must have the shape of q0")
    if H is not None and (H.dtype != torch.float64 or tuple(H.shape) != tuple(hshape)
                          or not H.is_contiguous()):
        raise ValueError(f"H must be contiguous float64 of shape {tuple(hshape)}")
    return q1, p1, H


def gs_shoot(q0, p0, prm: Params, method=GS_EXACT, with_energy=True, ws=None, out=None):
    """Forward-Euler shooting; returns (q1, p1, H) with H float64 (nt+1,) or None.
    `out` = (q1, p1, H or None) writes into the caller's buffers."""
    _pts(q0, torch.float32, "q0")
    _pts(p0, torch.float32, "p0")
    n = q0.shape[0]
    q1, p1, H = _outputs(out, q0, (prm.nt + 1,), with_energy)
    if ws is None:
        ws = _workspace(n, prm, method, GS_OP_SHOOT, q0.device)
    _check(lib().gs_shoot(_ptr(q0), _ptr(p0), n, ctypes.byref(prm), method, _ptr(q1),
                          _ptr(p1), _ptr(H), _ptr(ws), ws.numel(), _stream(q0.device)))
    return q1, p1, H


def gs_shoot_f64(q0, p0, prm: Params, with_energy=True):
    _pts(q0, torch.float64, "q0")
    _pts(p0, torch.float64, "p0")
    n = q0.shape[0]
    q1, p1 = torch.empty_like(q0), torch.empty_like(p0)
    H = torch.zeros(prm.nt + 1, dtype=torch.float64, device=q0.device) if with_energy else None
    pr = Params.from_buffer_copy(prm)
    pr.flags |= GS_FLAG_F64
    ws = _workspace(n, pr, GS_EXACT, GS_OP_SHOOT, q0.device)
    _check(lib().gs_shoot_f64(_ptr(q0), _ptr(p0), n, ctypes.byref(prm), _ptr(q1), _ptr(p1),
                              _ptr(H), _ptr(ws), ws.numel(), _stream(q0.device)))
    return q1, p1, H


def _grad_outputs(out, q0, nobj):
    """(objective, grad): the caller's buffers `out`, checked, or new ones.
    Passing the same buffers again lets a GS_FLAG_GRAPH call replay."""
    if out is None:
        return torch.zeros(nobj, dtype=torch.float64, device=q0.device), torch.empty_like(q0)
    obj, grad = out
    _pts(grad, torch.float32, "grad")
    if grad.shape != q0.shape:
        raise ValueError("grad must have the shape of q0")
    if obj.dtype != torch.float64 or obj.numel() != nobj or not obj.is_contiguous():
        raise ValueError(f"objective must be contiguous float64 with {nobj} entries")
    return obj, grad


def gs_shoot_adjoint(q0, p0, target, prm: Params, method=GS_EXACT, lam=0.01, ckpt_every=8,
                     ws=None, out=None):
    """Objective E(p0) (float64 scalar tensor) and dE/dp0 (float32 (n, 3)).
    `out` = (objective (1,) float64, grad) writes into the caller's buffers."""
    _pts(q0, torch.float32, "q0")
    _pts(p0, torch.float32, "p0")
    _pts(target, torch.float32, "target")
    n = q0.shape[0]
    obj, grad = _grad_outputs(out, q0, 1)
    if ws is None:
        nbytes = lib().gs_adjoint_workspace_bytes(n, ctypes.byref(prm), method, int(ckpt_every))
        if nbytes == 0:
            raise GsError(-1, "invalid arguments for gs_adjoint_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=q0.device)
    _check(lib().gs_shoot_adjoint(_ptr(q0), _ptr(p0), _ptr(target), n, ctypes.byref(prm),
                                  method, float(lam), int(ckpt_every), _ptr(obj), _ptr(grad),
                                  _ptr(ws), ws.numel(), _stream(q0.device)))
    return obj[0], grad


def gs_field(x, q, p, prm: Params):
    """Velocity field of eq. (3) at points x; float32 (m, 3)."""
    _pts(x, torch.float32, "x")
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    v = torch.empty_like(x)
    nbytes = lib().gs_field_workspace_bytes(x.shape[0], q.shape[0], ctypes.byref(prm))
    if nbytes == 0:
        raise GsError(-1, "invalid arguments for gs_field_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    _check(lib().gs_field(_ptr(x), x.shape[0], _ptr(q), _ptr(p), q.shape[0], ctypes.byref(prm),
                          _ptr(v), _ptr(ws), ws.numel(), _stream(x.device)))
    return v


def _offsets(offsets):
    """Host int64 array of the set boundaries (list, numpy array or CPU tensor)."""
    vals = [int(x) for x in (offsets.tolist() if hasattr(offsets, "tolist") else offsets)]
    if len(vals) < 2:
        raise GsError(-1, "offsets needs at least two entries")
    return (ctypes.c_int64 * len(vals))(*vals), len(vals) - 1


def gs_batch_workspace_bytes(offsets, prm: Params, method=GS_EXACT, op=GS_OP_RHS) -> int:
    off, nsub = _offsets(offsets)
    return int(lib().gs_batch_workspace_bytes(off, nsub, ctypes.byref(prm), method, op))


def _batch_workspace(off, nsub, prm, method, op, dev):
    nbytes = lib().gs_batch_workspace_bytes(off, nsub, ctypes.byref(prm), method, op)
    if nbytes == 0:
        raise GsError(-1, "invalid arguments for gs_batch_workspace_bytes: "
                          + lib().gs_last_error().decode())
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)


def gs_rhs_batch(q, p, offsets, prm: Params, method=GS_EXACT, ws=None, return_ws=False):
    """(dq, dp) of every set of a batch (rows offsets[s]..offsets[s+1] are set s)."""
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    off, nsub = _offsets(offsets)
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    if ws is None:
        ws = _batch_workspace(off, nsub, prm, method, GS_OP_RHS, q.device)
    _check(lib().gs_rhs_batch(_ptr(q), _ptr(p), off, nsub, ctypes.byref(prm), method, _ptr(dq),
                              _ptr(dp), _ptr(ws), ws.numel(), _stream(q.device)))
    return (dq, dp, ws) if return_ws else (dq, dp)


def gs_shoot_batch(q0, p0, offsets, prm: Params, method=GS_EXACT, with_energy=True, ws=None,
                   return_ws=False, out=None):
    """Shooting of every set of a batch; returns (q1, p1, H) with H float64
    (nsub, nt + 1) or None.  `out` = (q1, p1, H or None) as in gs_shoot."""
    _pts(q0, torch.float32, "q0")
    _pts(p0, torch.float32, "p0")
    off, nsub = _offsets(offsets)
    q1, p1, H = _outputs(out, q0, (nsub, prm.nt + 1), with_energy)
    if ws is None:
        ws = _batch_workspace(off, nsub, prm, method, GS_OP_SHOOT, q0.device)
    _check(lib().gs_shoot_batch(_ptr(q0), _ptr(p0), off, nsub, ctypes.byref(prm), method,
                                _ptr(q1), _ptr(p1), _ptr(H), _ptr(ws), ws.numel(),
                                _stream(q0.device)))
    return (q1, p1, H, ws) if return_ws else (q1, p1, H)


def gs_shoot_adjoint_batch(q0, p0, target, offsets, prm: Params, method=GS_EXACT, lam=0.01,
                           ckpt_every=8, ws=None, out=None):
    """Per-set objectives E_s (float64 (nsub,)) and dE_s/dp0 of every set
    (float32 (n, 3), rows of set s from its own objective).  `out` =
    (objectives, grad) writes into the caller's buffers."""
    _pts(q0, torch.float32, "q0")
    _pts(p0, torch.float32, "p0")
    _pts(target, torch.float32, "target")
    off, nsub = _offsets(offsets)
    obj, grad = _grad_outputs(out, q0, nsub)
    if ws is None:
        nbytes = lib().gs_adjoint_batch_workspace_bytes(off, nsub, ctypes.byref(prm), method,
                                                        int(ckpt_every))
        if nbytes == 0:
            raise GsError(-1, "invalid arguments for gs_adjoint_batch_workspace_bytes: "
                              + lib().gs_last_error().decode())
        ws = torch.empty(nbytes, dtype=torch.uint8, device=q0.device)
    _check(lib().gs_shoot_adjoint_batch(_ptr(q0), _ptr(p0), _ptr(target), off, nsub,
                                        ctypes.byref(prm), method, float(lam), int(ckpt_every),
                                        _ptr(obj), _ptr(grad), _ptr(ws), ws.numel(),
                                        _stream(q0.device)))
    return obj, grad


def gs_autotune_leaf_cap(q, p, prm: Params, offsets=None, ws=None):
    """Picks the fastest Barnes-Hut leaf_cap for these inputs; returns a copy
    of prm with it set, and the time of one RHS (ms) at that setting."""
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    off, nsub = _offsets([0, q.shape[0]] if offsets is None else offsets)
    out = Params.from_buffer_copy(prm)
    if ws is None:
        ws = _batch_workspace(off, nsub, out, GS_BH, GS_OP_RHS, q.device)
    ms = ctypes.c_double(0.0)
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    _check(lib().gs_autotune_leaf_cap(_ptr(q), _ptr(p), off, nsub, ctypes.byref(out), _ptr(dq),
                                      _ptr(dp), _ptr(ws), ws.numel(), _stream(q.device),
                                      ctypes.byref(ms)))
    return out, ms.value


def gs_autotune_exact(q, p, prm: Params, offsets=None, ws=None):
    """Picks the fastest exact_items for these inputs (exact FP32 path);
    returns a copy of prm with it set, and the time of one RHS (ms)."""
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    off, nsub = _offsets([0, q.shape[0]] if offsets is None else offsets)
    out = Params.from_buffer_copy(prm)
    if ws is None:
        big = Params.from_buffer_copy(prm)
        big.exact_items = 49152  # the largest candidate needs the largest workspace
        ws = _batch_workspace(off, nsub, big, GS_EXACT, GS_OP_RHS, q.device)
    ms = ctypes.c_double(0.0)
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    _check(lib().gs_autotune_exact(_ptr(q), _ptr(p), off, nsub, ctypes.byref(out), _ptr(dq),
                                   _ptr(dp), _ptr(ws), ws.numel(), _stream(q.device),
                                   ctypes.byref(ms)))
    return out, ms.value


def gs_tree_export(q, p, prm: Params) -> dict:
    """The octree gs_rhs_bh builds for (q, p), copied to the host (numpy
    arrays): sorted keys, permutation and per-node records."""
    import numpy as np
    _pts(q, torch.float32, "q")
    _pts(p, torch.float32, "p")
    n = q.shape[0]
    ws = _workspace(n, prm, GS_BH, GS_OP_RHS, q.device)
    keys = np.zeros(n, np.uint64)
    perm = np.zeros(n, np.uint32)
    nn = ctypes.c_int64(0)
    args = [_ptr(q), _ptr(p), n, ctypes.byref(prm), _ptr(ws), ws.numel(), _stream(q.device)]
    _check(lib().gs_tree_export(*args, 0, ctypes.byref(nn), keys.ctypes.data, perm.ctypes.data,
                                None, None, None, None, None))
    m = nn.value
    start, count, first, nchild = (np.zeros(m, np.int32) for _ in range(4))
    stats = np.zeros((m, 13))
    _check(lib().gs_tree_export(*args, m, ctypes.byref(nn), keys.ctypes.data, perm.ctypes.data,
                                start.ctypes.data, count.ctypes.data, first.ctypes.data,
                                nchild.ctypes.data, stats.ctypes.data))
    return {"keys": keys, "perm": perm, "start": start, "count": count, "first": first,
            "nchild": nchild, "C": stats[:, 0:3], "P": stats[:, 3:6], "lo": stats[:, 6:9],
            "hi": stats[:, 9:12], "s2": stats[:, 12]}


def gs_get_status(ws) -> int:
    return int(lib().gs_get_status(_ptr(ws), _stream(ws.device)))


def gs_bh_counters(ws) -> dict:
    out = (ctypes.c_int64 * 8)()
    _check(lib().gs_bh_counters(_ptr(ws), _stream(ws.device), out))
    return {"pairs": out[0], "monopoles": out[1], "visits": out[2], "nodes": out[3],
            "wave_leaf_steps": out[4], "wave_node_decisions": out[5], "max_wave_work": out[6],
            "max_decide_wave_nodes": out[7]}


def gs_kernel_timing(enable: bool):
    _check(lib().gs_kernel_timing(1 if enable else 0))


KINDS = ("exact", "traverse", "adjoint", "tree", "exact_v", "traverse_v")


def gs_kernel_timing_read() -> dict:
    c = (ctypes.c_int64 * len(KINDS))()
    ms = (ctypes.c_double * len(KINDS))()
    _check(lib().gs_kernel_timing_read(c, ms))
    return {k: {"launches": int(c[i]), "ms": float(ms[i])} for i, k in enumerate(KINDS)}


@dataclass
class Shot:
    q1: torch.Tensor
    p1: torch.Tensor
    H: torch.Tensor | None


def shoot(q0, p0, sigma, nt=40, method="exact", theta=0.5, leaf_cap=1, cutoff_sigmas=3.0):
    """Convenience wrapper: shoot FP32 (or FP64 exact) point sets."""
    prm = params(sigma, nt=nt, theta=theta, leaf_cap=leaf_cap, cutoff_sigmas=cutoff_sigmas)
    if q0.dtype == torch.float64:
        if method != "exact":
            raise GsError(-5, "FP64 shooting is exact only")
        return Shot(*gs_shoot_f64(q0, p0, prm))
    return Shot(*gs_shoot(q0, p0, prm, GS_EXACT if method == "exact" else GS_BH))


INF = math.inf


class ShootLoss(torch.autograd.Function):
    """E(p0) = |q(1) - target|^2 / n + lam <p0, K(q0) p0> as a differentiable
    function of p0 (float32 (n, 3)); the backward pass returns the
    gradient computed by gs_shoot_adjoint's discrete adjoint."""

    @staticmethod
    def forward(ctx, p0, q0, target, sigma, nt=40, lam=0.01, method="exact", theta=0.5,
                leaf_cap=1, ckpt_every=8):
        prm = params(sigma, nt=nt, theta=theta, leaf_cap=leaf_cap)
        m = GS_EXACT if method == "exact" else GS_BH
        e, g = gs_shoot_adjoint(q0.contiguous(), p0.detach().contiguous(), target.contiguous(),
                                prm, m, lam, ckpt_every)
        ctx.save_for_backward(g)
        return e.clone()

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (grad_out.to(g.dtype) * g, None, None, None, None, None, None, None, None, None)


def shoot_loss(p0, q0, target, sigma, **kw):
    return ShootLoss.apply(p0, q0, target, sigma, *[kw.get(k, d) for k, d in (
        ("nt", 40), ("lam", 0.01), ("method", "exact"), ("theta", 0.5), ("leaf_cap", 1),
        ("ckpt_every", 8))])
