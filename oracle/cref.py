"""ctypes wrapper of the C oracle (oracle/c/mpref.c).

TEST INFRASTRUCTURE ONLY (see oracle/mpnum.py).  Matrices are numpy uint32
arrays in the plane layout (L + 2, rows, ld).
"""

import ctypes
import os

import numpy as np

from .c import build as _build

ALGO = {"simple": 0, "block": 1, "strassen": 2, "winograd": 3}
POLICY = {"peel": 0, "pad": 1, "mixed": 2}

_libs = {}
NARROW_MAXL = 48


def lib(p=None, residual=False):
    """The narrow build when values of p bits (and, for a residual, 2p + 64
    bits) fit its 48 limbs, else the wide build (656 limbs)."""
    need = 0 if p is None else (2 * (p // 32) + 2 if residual else p // 32)
    wide = need > NARROW_MAXL
    if wide not in _libs:
        # MPREF_SANITIZE=1 loads the address / undefined-behaviour instrumented
        # builds (the process must preload the sanitizer runtime)
        path = _build.build(wide=wide, sanitize=os.environ.get("MPREF_SANITIZE") == "1")
        L = ctypes.CDLL(path)
        i64, i32, u32p, i32p = ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int32)
        L.ref_gemm.argtypes = [i64, i64, i64, i32, i32, i64, i32, i64,
                               u32p, i64, i64, u32p, i64, i64, u32p, i64, i64]
        L.ref_gemm.restype = i32
        L.ref_scalar.argtypes = [i32, i32, u32p, u32p, u32p]
        L.ref_scalar.restype = i32
        L.ref_lu.argtypes = [i64, i32, i64, i32, i64, i32, u32p, i64, i64, i32p, i32p]
        L.ref_lu.restype = i32
        L.ref_lu_ex.argtypes = [i64, i32, i64, i32, i64, i32, i32, u32p, i64, i64, i32p, i32p]
        L.ref_lu_ex.restype = i32
        L.ref_lu_solve.argtypes = [i64, i32, u32p, i64, i64, i32p, u32p, i64]
        L.ref_lu_solve.restype = i32
        L.ref_lu_residual.argtypes = [i64, i32, u32p, i64, i64, u32p, i64, i64, i32p,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.ref_lu_residual.restype = i32
        L.ref_threads.argtypes = [i32]
        L.ref_threads.restype = i32
        _libs[wide] = L
    return _libs[wide]


def _p(a):
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def threads(t=0):
    """Set the OpenMP thread count (t > 0); returns the count in use."""
    lib(10240).ref_threads(int(t))
    return lib().ref_threads(int(t))


def gemm(A, B, p, algo="simple", cutoff=32, policy="peel", block_size=16, m=None, l=None, n=None):
    """C = AB by the C oracle; A, B in the plane layout (ld = array width)."""
    m = A.shape[1] if m is None else m
    l = A.shape[2] if l is None else l
    n = B.shape[2] if n is None else n
    L = p // 32
    C = np.zeros((L + 2, m, max(n, 1)), dtype=np.uint32)
    rc = lib(p).ref_gemm(m, l, n, p, ALGO[algo], cutoff, POLICY[policy], block_size,
                        _p(A), A.shape[2], A.shape[1] * A.shape[2],
                        _p(B), B.shape[2], B.shape[1] * B.shape[2],
                        _p(C), C.shape[2], C.shape[1] * C.shape[2])
    if rc:
        raise RuntimeError("ref_gemm failed: %d" % rc)
    return C


def scalar(op, p, x, y):
    """One scalar op on (L + 2)-word records; op in mul/add/sub/div."""
    code = {"mul": 0, "add": 1, "sub": 2, "div": 3}[op]
    r = np.zeros(p // 32 + 2, dtype=np.uint32)
    rc = lib(p).ref_scalar(code, p, _p(np.ascontiguousarray(x)), _p(np.ascontiguousarray(y)), _p(r))
    if rc:
        raise RuntimeError("ref_scalar failed: %d" % rc)
    return r


def lu(A, p, panel=64, algo="winograd", cutoff=32, policy="peel", pivot=True):
    """Returns (LU planes, piv, info); A is not modified.  pivot=False: the
    paper's LU without row exchanges (piv is then the identity)."""
    n = A.shape[1]
    F = np.ascontiguousarray(A.copy())
    piv = np.zeros(n, dtype=np.int32)
    info = ctypes.c_int32(0)
    rc = lib(p).ref_lu_ex(n, p, panel, ALGO[algo], cutoff, POLICY[policy], 1 if pivot else 0, _p(F), F.shape[2],
                         F.shape[1] * F.shape[2], piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         ctypes.byref(info))
    if rc:
        raise RuntimeError("ref_lu failed: %d" % rc)
    return F, piv, info.value


def lu_solve(F, piv, b, p):
    n = F.shape[1]
    x = np.ascontiguousarray(b.copy())
    rc = lib(p).ref_lu_solve(n, p, _p(F), F.shape[2], F.shape[1] * F.shape[2],
                            np.ascontiguousarray(piv, dtype=np.int32).ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            _p(x), x.shape[1] * x.shape[2])
    if rc:
        raise RuntimeError("ref_lu_solve failed: %d" % rc)
    return x


def lu_residual(A, F, piv, p):
    """||PA - LU||_inf / ||A||_inf as (mantissa, exp2) -> returns log2 and value."""
    import math
    n = A.shape[1]
    m = ctypes.c_double(0.0)
    e = ctypes.c_int64(0)
    rc = lib(p, residual=True).ref_lu_residual(n, p, _p(A), A.shape[2], A.shape[1] * A.shape[2],
                               _p(F), F.shape[2], F.shape[1] * F.shape[2],
                               np.ascontiguousarray(piv, dtype=np.int32).ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.byref(m), ctypes.byref(e))
    if rc:
        raise RuntimeError("ref_lu_residual failed: %d" % rc)
    if m.value == 0.0:
        return float("-inf"), 0.0
    l2 = math.log2(m.value) + e.value
    return l2, (math.ldexp(m.value, int(e.value)) if e.value > -1000 else 0.0)
