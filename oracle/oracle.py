"""ctypes front end of the double-precision CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module; the GPU library and
its Python binding never do.  Every function takes and returns float64 numpy
arrays of shape (n, 3); float32 inputs are promoted exactly.

Paper: Wang, Xie, Yushkevich, Gee, "Barnes-Hut Approximation for Point Set
Geodesic Shooting" (arXiv:1907.04834).  The readings of the paper that the
oracle takes are listed in the header of ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# GS_ORACLE_LIB selects another build (the sanitized one of the sanitizer
# checks, see build_sanitized); by default the in-tree liboracle.so.
_ALT = os.environ.get("GS_ORACLE_LIB")
_LIB = _ALT or os.path.join(_HERE, "liboracle.so")

# No FMA contraction, no fast-math: every operation is the IEEE double one.
GCC_CMD = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (when missing or stale, or if forced)."""
    if _ALT:
        return _LIB
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
    if force or stale:
        subprocess.run(GCC_CMD, check=True)
    return _LIB


CLANG = "/opt/rocm/lib/llvm/bin/clang"


def build_sanitized(out: str) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (clang, the runtime of the host-sanitized GPU library build; serial:
    without OpenMP), for the sanitizer checks of the test suite."""
    subprocess.run([CLANG, "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-shared-libasan", "-Wno-unknown-pragmas",
                    "-fPIC", "-shared", "-o", out, _SRC, "-lm"], check=True)
    return out


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U64 = ctypes.POINTER(ctypes.c_uint64)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_i64, _i32, _dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_rhs_exact.argtypes = [_i64, _D, _D, _dbl, _D, _D]
        L.or_field_exact.argtypes = [_i64, _D, _i64, _D, _D, _dbl, _D]
        L.or_rhs_exact_rows.argtypes = [_i64, _I64, _i64, _D, _D, _dbl, _D, _D]
        L.or_energy.argtypes = [_i64, _D, _D]
        L.or_energy.restype = _dbl
        L.or_rhs_bh.argtypes = [_i64, _D, _D, _dbl, _dbl, _dbl, _i32, _D, _D,
                                _I64, _D, _D]
        L.or_tree_dump.argtypes = [_i64, _D, _D, _i32, _I64, _i64, _I32, _U64,
                                   _I64, _I32, _I32, _D]
        L.or_tree_dump.restype = _i64
        L.or_int_coords.argtypes = [_i64, _D, _U32]
        L.or_shoot.argtypes = [_i64, _D, _D, _dbl, _i32, _i32, _dbl, _dbl, _i32,
                               _D, _D, _D]
        L.or_adjoint_rhs.argtypes = [_i64, _D, _D, _D, _D, _dbl, _i32, _dbl, _dbl,
                                     _i32, _D, _D]
        L.or_objective_grad.argtypes = [_i64, _D, _D, _D, _dbl, _i32, _dbl, _i32,
                                        _dbl, _dbl, _i32, _D]
        L.or_objective_grad.restype = _dbl
        L.or_version.restype = ctypes.c_char_p
        L.or_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [_i32]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def _d(x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return x, x.ctypes.data_as(_D)


def _out(n):
    x = np.zeros((n, 3), dtype=np.float64)
    return x, x.ctypes.data_as(_D)


def _method(method) -> int:
    return {"exact": 0, "bh": 1, 0: 0, 1: 1}[method]


def rhs_exact(q, p, sigma):
    """(v, a) of the exact right-hand side (all pairs, self term included)."""
    q, qp = _d(q)
    p, pp = _d(p)
    n = q.shape[0]
    v, vp = _out(n)
    a, ap = _out(n)
    lib().or_rhs_exact(n, qp, pp, sigma, vp, ap)
    return v, a


def rhs_exact_rows(idx, q, p, sigma):
    """Exact RHS for targets idx only (all sources); returns (v, a) rows."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    q, qp = _d(q)
    p, pp = _d(p)
    m = idx.shape[0]
    v, vp = _out(m)
    a, ap = _out(m)
    lib().or_rhs_exact_rows(m, idx.ctypes.data_as(_I64), q.shape[0], qp, pp,
                            sigma, vp, ap)
    return v, a


def field_exact(x, q, p, sigma):
    """Velocity field of eq. (3) at points x."""
    x, xp = _d(x)
    q, qp = _d(q)
    p, pp = _d(p)
    v, vp = _out(x.shape[0])
    lib().or_field_exact(x.shape[0], xp, q.shape[0], qp, pp, sigma, vp)
    return v


def energy(p, v) -> float:
    p, pp = _d(p)
    v, vp = _d(v)
    return lib().or_energy(p.shape[0], pp, vp)


def rhs_bh(q, p, sigma, theta, kappa=3.0, leaf_cap=1, bounds=False):
    """Barnes-Hut RHS.  Returns (v, a, counters) and, with bounds=True, the
    per-target a-priori error bounds (bound_v, bound_a) as well.  counters is
    a dict with exact pairs, monopoles and node visits summed over targets."""
    q, qp = _d(q)
    p, pp = _d(p)
    n = q.shape[0]
    v, vp = _out(n)
    a, ap = _out(n)
    cnt = np.zeros(3, dtype=np.int64)
    bv = np.zeros(n)
    ba = np.zeros(n)
    lib().or_rhs_bh(n, qp, pp, sigma, kappa, theta, leaf_cap, vp, ap,
                    cnt.ctypes.data_as(_I64), bv.ctypes.data_as(_D),
                    ba.ctypes.data_as(_D))
    c = {"pairs": int(cnt[0]), "monopoles": int(cnt[1]), "visits": int(cnt[2])}
    if bounds:
        return v, a, c, bv, ba
    return v, a, c


def shoot(q0, p0, sigma, nt, method="exact", theta=0.5, kappa=3.0, leaf_cap=1):
    """Forward-Euler shooting over [0, 1].  Returns (q1, p1, H[0..nt])."""
    q0, qp = _d(q0)
    p0, pp = _d(p0)
    n = q0.shape[0]
    q1, q1p = _out(n)
    p1, p1p = _out(n)
    H = np.zeros(nt + 1)
    lib().or_shoot(n, qp, pp, sigma, nt, _method(method), kappa, theta, leaf_cap,
                   q1p, p1p, H.ctypes.data_as(_D))
    return q1, p1, H


def adjoint_rhs(q, p, alpha, beta, sigma, method="exact", theta=0.5, kappa=3.0,
                leaf_cap=1):
    """One backward-stage product J(q, p)^T (alpha, beta) -> (g_q, g_p)."""
    q, qp = _d(q)
    p, pp = _d(p)
    al, alp = _d(alpha)
    be, bep = _d(beta)
    n = q.shape[0]
    gq, gqp = _out(n)
    gp, gpp = _out(n)
    lib().or_adjoint_rhs(n, qp, pp, alp, bep, sigma, _method(method), kappa,
                         theta, leaf_cap, gqp, gpp)
    return gq, gp


def objective_grad(q0, p0, y, sigma, nt, lam, method="exact", theta=0.5,
                   kappa=3.0, leaf_cap=1, grad=True):
    """E(p0) = |q(1) - y|^2 / n + lam <p0, K(q0) p0> and (optionally) dE/dp0."""
    q0, qp = _d(q0)
    p0, pp = _d(p0)
    y, yp = _d(y)
    n = q0.shape[0]
    g, gp = _out(n)
    e = lib().or_objective_grad(n, qp, pp, yp, sigma, nt, lam, _method(method),
                                kappa, theta, leaf_cap, gp if grad else None)
    return (e, g) if grad else e


def tree_dump(q, p, leaf_cap=1, order=None):
    """Nodes of the recursive-insertion octree as a dict of arrays."""
    q, qp = _d(q)
    p, pp = _d(p)
    n = q.shape[0]
    L = lib()
    op = None
    if order is not None:
        order = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
        op = order.ctypes.data_as(_I64)
    m = L.or_tree_dump(n, qp, pp, leaf_cap, op, 0, None, None, None, None, None,
                       None)
    level = np.zeros(m, dtype=np.int32)
    prefix = np.zeros(m, dtype=np.uint64)
    count = np.zeros(m, dtype=np.int64)
    leaf = np.zeros(m, dtype=np.int32)
    nch = np.zeros(m, dtype=np.int32)
    st = np.zeros((m, 12))
    L.or_tree_dump(n, qp, pp, leaf_cap, op, m, level.ctypes.data_as(_I32),
                   prefix.ctypes.data_as(_U64), count.ctypes.data_as(_I64),
                   leaf.ctypes.data_as(_I32), nch.ctypes.data_as(_I32),
                   st.ctypes.data_as(_D))
    return {"level": level, "prefix": prefix, "count": count, "leaf": leaf,
            "nchild": nch, "P": st[:, 0:3], "C": st[:, 3:6], "lo": st[:, 6:9],
            "hi": st[:, 9:12]}


def int_coords(q):
    """Integer octree coordinates (21 bits per axis) of every point."""
    q, qp = _d(q)
    ic = np.zeros((q.shape[0], 3), dtype=np.uint32)
    lib().or_int_coords(q.shape[0], qp, ic.ctypes.data_as(_U32))
    return ic


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Sets the OpenMP threads of the oracle's parallel loops (for timing)."""
    lib().or_set_threads(int(n))


def version() -> str:
    return lib().or_version().decode()
