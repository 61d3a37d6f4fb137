"""Python binding of libmpgemm (include/mpgemm.h): argument marshalling only.

Matrices are torch tensors on the GPU in the library's plane layout: shape
(L + 2, rows, ld), dtype int32 (the words are reinterpreted as uint32 by the
library), last dimension contiguous; ld = stride(1), plane stride = stride(0).
Every function here forwards to the C function of the same name on torch's
current stream.  If the library is missing or cannot be loaded the import of
this module fails: there is no fallback.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmpgemm.so")

SIMPLE, BLOCK, STRASSEN, WINOGRAD, AUTO = 0, 1, 2, 3, 4
ALGOS = {"simple": SIMPLE, "block": BLOCK, "strassen": STRASSEN, "winograd": WINOGRAD, "auto": AUTO}
PEEL, PAD, MIXED = 0, 1, 2
POLICIES = {"peel": PEEL, "pad": PAD, "mixed": MIXED}
LEAF_SIMPLE, LEAF_BLOCK = 0, 1

MP_OK = 0


class MPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libmpgemm error %d: %s" % (code, msg))
        self.code = code


def _load():
    # torch first: its HIP runtime is then the one the library binds to (its
    # libamdhip64 dependency resolves to the copy torch already loaded), so
    # torch's allocations and streams are valid inside the library
    import torch  # noqa: F401
    if not os.path.exists(LIBPATH):
        raise ImportError("libmpgemm.so is not built (run python -m paper_1410_1599_amd.build)")
    lib = ctypes.CDLL(LIBPATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    dp, i32p, i64p = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)
    mat = [vp, i64, i64]
    sig = {
        "mp_set_stream": ([vp], i32),
        "mp_last_error": ([], ctypes.c_char_p),
        "mp_version": ([], i32),
        "mp_set_policy": ([i32, i32], i32),
        "mp_gemm": ([i64, i64, i64, i32, i32, i32] + mat * 3, i32),
        "mp_gemm_ex": ([i64, i64, i64, i32, i32, i32, i32, i32] + mat * 3, i32),
        "mp_gemm_noalloc": ([i64, i64, i64, i32, i32, i32] + mat * 3, i32),
        "mp_add": ([i64, i64, i32] + mat * 3, i32),
        "mp_sub": ([i64, i64, i32] + mat * 3, i32),
        "mp_mul_ew": ([i64, i64, i32] + mat * 3, i32),
        "mp_div_ew": ([i64, i64, i32] + mat * 3, i32),
        "mp_plan_info": ([i64, i64, i64, i32, i32, i32, i32, i32p, dp, dp, i64p, i64p], i32),
        "mp_lu": ([i64, i32, vp, i64, i64, vp, i32p], i32),
        "mp_lu_ex": ([i64, i32, vp, i64, i64, vp, i32p, i32, i32, i32, i32], i32),
        "mp_lu_nopivot": ([i64, i32, vp, i64, i64, vp, i32p, i32, i32, i32, i32], i32),
        "mp_lu_solve": ([i64, i32, vp, i64, i64, vp, vp, i64], i32),
        "mp_release_workspace": ([], i32),
        "mp_profile": ([i32], i32),
        "mp_gemm_slice": ([i64, i64, i64, i32, i32] + mat * 3 + [i32p], i32),
        "mp_set_slice_guard": ([i32], i32),
        "mp_slice_last": ([i32p], i32),
        "mp_set_graph_mode": ([i32], i32),
        "mp_fill_uniform": ([i64, i64, i32, vp, i64, i64, ctypes.c_uint64], i32),
        "mp_gemm_batched": ([i32, i64p, i64p, i64p, i32, i32, i32] + [ctypes.POINTER(vp), i64p, i64p] * 3, i32),
        "mp_tune": ([i64, i64, i64, i32, i32, i32p, i32p, i32p, ctypes.POINTER(ctypes.c_float)], i32),
        "mp_auto_choice": ([i64, i64, i64, i32, i32p, i32p, i32p], i32),
        "mp_auto_launch": ([i64, i64, i64, i32, i32p, i32p, i32p, i32p, i32p], i32),
        "mp_set_launch": ([i32, i32], i32),
        "mp_tune_save": ([ctypes.c_char_p], i32),
        "mp_tune_load": ([ctypes.c_char_p], i32),
        "mp_lu_async": ([i64, i32, vp, i64, i64, vp, vp, i32, i32, i32, i32], i32),
        "mp_profile_read": ([i32, i32p, i32p, i32p, dp, i64p, ctypes.POINTER(ctypes.c_float)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def last_error():
    return lib.mp_last_error().decode()


def _check(rc):
    if rc != MP_OK:
        raise MPError(rc, last_error())
    return rc


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mat(t):
    """(pointer, ld, plane stride) of a plane-layout tensor."""
    if t is None:
        return (None, 0, 0)
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("matrix tensors are (L + 2, rows, ld) with a contiguous last dimension")
    return (ctypes.c_void_p(t.data_ptr()), t.stride(1), t.stride(0))


def nlimbs(prec):
    return prec // 32


# ----------------------------------------------------------------- tensors

def to_device(planes, device="cuda"):
    """numpy uint32 planes (L + 2, rows, ld) -> int32 torch tensor on the GPU."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(planes).view(np.int32)).to(device)


def to_host(t):
    """torch plane tensor -> numpy uint32 planes."""
    return t.detach().cpu().contiguous().numpy().view(np.uint32)


def empty(rows, cols, prec, device="cuda"):
    import torch
    return torch.zeros((nlimbs(prec) + 2, rows, cols), dtype=torch.int32, device=device)


# ----------------------------------------------------------------- the C functions

def mp_set_stream(stream=None):
    return _check(lib.mp_set_stream(stream if stream is not None else _stream()))


def mp_set_policy(odd_policy=PEEL, leaf=LEAF_SIMPLE):
    return _check(lib.mp_set_policy(int(odd_policy), int(leaf)))


def mp_gemm(m, l, n, prec, algo, cutoff, A, B, C):
    mp_set_stream()
    return _check(lib.mp_gemm(m, l, n, prec, int(algo), int(cutoff), *_mat(A), *_mat(B), *_mat(C)))


def mp_gemm_noalloc(m, l, n, prec, algo, cutoff, A, B, C):
    mp_set_stream()
    return _check(lib.mp_gemm_noalloc(m, l, n, prec, int(algo), int(cutoff), *_mat(A), *_mat(B), *_mat(C)))


def mp_gemm_ex(m, l, n, prec, algo, cutoff, policy, leaf, A, B, C):
    mp_set_stream()
    return _check(lib.mp_gemm_ex(m, l, n, prec, int(algo), int(cutoff), int(policy), int(leaf),
                                 *_mat(A), *_mat(B), *_mat(C)))


def _ew(fn, m, n, prec, A, B, C):
    mp_set_stream()
    return _check(fn(m, n, prec, *_mat(A), *_mat(B), *_mat(C)))


def mp_add(m, n, prec, A, B, C):
    return _ew(lib.mp_add, m, n, prec, A, B, C)


def mp_sub(m, n, prec, A, B, C):
    return _ew(lib.mp_sub, m, n, prec, A, B, C)


def mp_mul_ew(m, n, prec, A, B, C):
    return _ew(lib.mp_mul_ew, m, n, prec, A, B, C)


def mp_div_ew(m, n, prec, A, B, C):
    return _ew(lib.mp_div_ew, m, n, prec, A, B, C)


def mp_plan_info(m, l, n, prec, algo, cutoff, policy=PEEL):
    d = ctypes.c_int(0)
    nm, na = ctypes.c_double(0), ctypes.c_double(0)
    ws, nl = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib.mp_plan_info(m, l, n, prec, int(algo), int(cutoff), int(policy), ctypes.byref(d),
                            ctypes.byref(nm), ctypes.byref(na), ctypes.byref(ws), ctypes.byref(nl)))
    return {"depth": d.value, "n_mul": nm.value, "n_addsub": na.value, "ws_bytes": ws.value, "n_launches": nl.value}


def mp_lu(n, prec, A, piv):
    mp_set_stream()
    info = ctypes.c_int(0)
    pa, lda, psa = _mat(A)
    _check(lib.mp_lu(n, prec, pa, lda, psa, ctypes.c_void_p(piv.data_ptr()), ctypes.byref(info)))
    return info.value


def mp_lu_ex(n, prec, A, piv, panel=64, algo=WINOGRAD, cutoff=32, policy=PEEL):
    mp_set_stream()
    info = ctypes.c_int(0)
    pa, lda, psa = _mat(A)
    _check(lib.mp_lu_ex(n, prec, pa, lda, psa, ctypes.c_void_p(piv.data_ptr()), ctypes.byref(info),
                        int(panel), int(algo), int(cutoff), int(policy)))
    return info.value


def mp_lu_nopivot(n, prec, A, piv, panel=64, algo=WINOGRAD, cutoff=32, policy=PEEL):
    """The paper's LU without row exchanges; piv receives the identity."""
    mp_set_stream()
    info = ctypes.c_int(0)
    pa, lda, psa = _mat(A)
    _check(lib.mp_lu_nopivot(n, prec, pa, lda, psa, ctypes.c_void_p(piv.data_ptr()), ctypes.byref(info),
                             int(panel), int(algo), int(cutoff), int(policy)))
    return info.value


def mp_lu_solve(n, prec, LU, piv, b):
    mp_set_stream()
    pa, lda, psa = _mat(LU)
    pb, _, psb = _mat(b)
    return _check(lib.mp_lu_solve(n, prec, pa, lda, psa, ctypes.c_void_p(piv.data_ptr()), pb, psb))


def mp_gemm_slice(m, l, n, prec, extra, A, B, C):
    """INT8-slice product; returns the windows (W_A, W_B) it used."""
    mp_set_stream()
    w = (ctypes.c_int * 2)()
    _check(lib.mp_gemm_slice(m, l, n, prec, int(extra), *_mat(A), *_mat(B), *_mat(C), w))
    return w[0], w[1]


def mp_set_slice_guard(guard_bits):
    return _check(lib.mp_set_slice_guard(int(guard_bits)))


def mp_slice_last():
    """(u0, diagonals, tiles recomputed, tiles, D) of the last slice product."""
    w = (ctypes.c_int * 5)()
    _check(lib.mp_slice_last(w))
    return tuple(int(x) for x in w)


def mp_release_workspace():
    return _check(lib.mp_release_workspace())


def mp_profile(enable):
    return _check(lib.mp_profile(1 if enable else 0))


def mp_profile_read(max_records=4096):
    """List of dicts (kind, op, L, units, ntiles, ms) of the recorded launches."""
    n = max_records
    kind, op, L = (ctypes.c_int * n)(), (ctypes.c_int * n)(), (ctypes.c_int * n)()
    units, nt, ms = (ctypes.c_double * n)(), (ctypes.c_int64 * n)(), (ctypes.c_float * n)()
    got = lib.mp_profile_read(n, kind, op, L, units, nt, ms)
    return [dict(kind=kind[i], op=op[i], L=L[i], units=units[i], ntiles=nt[i], ms=ms[i]) for i in range(min(got, n))]


def mp_set_graph_mode(enable):
    return _check(lib.mp_set_graph_mode(1 if enable else 0))


def mp_tune(m, l, n, prec, reps=2):
    mp_set_stream()
    a, c, lf = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    t = ctypes.c_float(0)
    _check(lib.mp_tune(m, l, n, prec, reps, ctypes.byref(a), ctypes.byref(c), ctypes.byref(lf), ctypes.byref(t)))
    return {"algo": a.value, "cutoff": c.value, "leaf": lf.value, "ms": t.value}


def mp_auto_choice(m, l, n, prec):
    a, c, lf = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(lib.mp_auto_choice(m, l, n, prec, ctypes.byref(a), ctypes.byref(c), ctypes.byref(lf)))
    return {"algo": a.value, "cutoff": c.value, "leaf": lf.value}


def mp_auto_launch(m, l, n, prec):
    v = [ctypes.c_int(0) for _ in range(5)]
    _check(lib.mp_auto_launch(m, l, n, prec, *[ctypes.byref(x) for x in v]))
    return dict(zip(("algo", "cutoff", "leaf", "tile_cols_log2", "persistent"), (x.value for x in v)))


def mp_set_launch(tile_cols_log2=0, persistent=0):
    return _check(lib.mp_set_launch(int(tile_cols_log2), int(persistent)))


def mp_tune_save(path):
    return _check(lib.mp_tune_save(path.encode()))


def mp_tune_load(path):
    got = lib.mp_tune_load(path.encode())
    if got < 0:
        raise MPError(got, last_error())
    return got


def mp_lu_async(n, prec, A, piv, info_dev, panel=64, algo=WINOGRAD, cutoff=32, policy=PEEL):
    mp_set_stream()
    pa, lda, psa = _mat(A)
    return _check(lib.mp_lu_async(n, prec, pa, lda, psa, ctypes.c_void_p(piv.data_ptr()),
                                  ctypes.c_void_p(info_dev.data_ptr()), int(panel), int(algo), int(cutoff), int(policy)))


def mp_gemm_batched(prec, algo, cutoff, As, Bs, Cs):
    """C_r := A_r B_r for every r, one grouped plan (lists of plane tensors)."""
    mp_set_stream()
    k = len(As)
    I64 = ctypes.c_int64 * k
    P = ctypes.c_void_p * k
    mats = [[_mat(t) for t in X] for X in (As, Bs, Cs)]
    m = I64(*[t.shape[1] for t in As])
    l = I64(*[t.shape[2] for t in As])
    n = I64(*[t.shape[2] for t in Bs])
    args = []
    for X in mats:
        args += [P(*[x[0] for x in X]), I64(*[x[1] for x in X]), I64(*[x[2] for x in X])]
    return _check(lib.mp_gemm_batched(k, m, l, n, prec, int(algo), int(cutoff), *args))


def mp_fill_uniform(rows, cols, prec, X, seed):
    mp_set_stream()
    px, ld, ps = _mat(X)
    return _check(lib.mp_fill_uniform(rows, cols, prec, px, ld, ps, ctypes.c_uint64(seed & ((1 << 64) - 1))))
