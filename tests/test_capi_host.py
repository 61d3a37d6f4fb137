"""Host-side checks of libmpgemm that need no GPU.

* the shared library loads and exports every function include/mpgemm.h
  declares;
* the planner's operation counts (mp_plan_info) equal the oracle's counts
  for every algorithm, policy and many shapes, and reproduce Table 1;
* every plan passes the library's own bounds validation;
* invalid arguments are rejected before anything touches the device.
"""

import ctypes
import itertools
import json
import os
import re

import pytest

from oracle import gemm as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mp():
    from paper_1410_1599_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=False)
    from paper_1410_1599_amd import mp as m
    return m


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "mpgemm.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return re.findall(r"^\s*(?:int|const char \*)\s*(mp_\w+)\s*\(", hdr, re.M)


def test_all_declared_symbols_exported(mp):
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(mp.LIBPATH)
    for n in names:
        assert hasattr(lib, n), n
    assert mp.lib.mp_version() == 1


@pytest.mark.parametrize("algo", ["strassen", "winograd"])
@pytest.mark.parametrize("policy", ["peel", "pad", "mixed"])
def test_plan_counts_equal_oracle_counts(mp, algo, policy):
    dims = [1, 3, 8, 31, 33, 64, 65, 100]
    for m, l, n in itertools.product(dims, repeat=3):
        for cut in (1, 4, 32):
            info = mp.mp_plan_info(m, l, n, 256, mp.ALGOS[algo], cut, mp.POLICIES[policy])
            assert (info["n_mul"], info["n_addsub"]) == G.op_counts(m, l, n, algo, cut, policy), (m, l, n, cut)
            assert info["depth"] == G.depth(m, l, n, cut, policy)


def test_plan_reproduces_table1(mp):
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_opcounts.json")))
    for row in gold["rows"]:
        n = row["n"]
        for algo in ("strassen", "winograd"):
            info = mp.mp_plan_info(n, n, n, 128, mp.ALGOS[algo], 32, mp.MIXED)
            assert round(info["n_mul"] / n ** 3, 3) == row[algo + "_mul"]
            assert round(info["n_addsub"] / n ** 3, 3) == row[algo + "_addsub"]


def test_workload_plans(mp):
    # the 2048 / cutoff 64 product: five levels, 7^5 leaves of 64^3, one
    # grouped leaf launch, three passes per level
    info = mp.mp_plan_info(2048, 2048, 2048, 256, mp.WINOGRAD, 64)
    assert info["depth"] == 5
    assert info["n_mul"] == 7 ** 5 * 64 ** 3
    assert info["n_launches"] == 5 * 3 + 1
    # 1023 peels at every level
    info = mp.mp_plan_info(1023, 1023, 1023, 256, mp.WINOGRAD, 64)
    assert info["depth"] == 4
    # simple and block: one launch, no workspace
    for a in (mp.SIMPLE, mp.BLOCK):
        info = mp.mp_plan_info(300, 200, 100, 512, a, 0)
        assert info["n_launches"] == 1 and info["ws_bytes"] == 0 and info["n_mul"] == 300 * 200 * 100


def test_argument_errors_without_device(mp):
    lib = mp.lib
    fake = ctypes.c_void_p(1 << 40)

    def gemm(m, l, n, prec, algo, cut, lda=None, ldb=None, ldc=None, C=None):
        lda = l if lda is None else lda
        ldb = n if ldb is None else ldb
        ldc = n if ldc is None else ldc
        return lib.mp_gemm(m, l, n, prec, algo, cut, fake, lda, m * lda, ctypes.c_void_p((1 << 40) + (1 << 36)),
                           ldb, l * ldb, C if C is not None else ctypes.c_void_p((1 << 40) + (2 << 36)), ldc, m * ldc)

    assert gemm(4, 4, 4, 100, 0, 0) == -2
    assert gemm(4, 4, 4, 256, 7, 0) == -1
    assert gemm(4, 4, 4, 256, 3, 0) == -1            # cutoff < 1
    assert gemm(-1, 4, 4, 256, 0, 0) == -1
    assert gemm(4, 4, 4, 256, 0, 0, lda=3) == -1      # ld < cols
    assert gemm(4, 4, 4, 256, 0, 0, C=fake) == -3     # C overlaps A
    assert gemm(1 << 31, 1, 1, 256, 0, 0) == -6
    assert "prec" in mp.last_error() or mp.last_error()
    assert lib.mp_plan_info(4, 4, 4, 96, 3, 4, 0, None, None, None, None, None) == -2
    assert lib.mp_set_policy(5, 0) == -1
    assert lib.mp_set_policy(0, 3) == -1
    info = ctypes.c_int(0)
    assert lib.mp_lu_ex(4, 256, fake, 4, 16, fake, ctypes.byref(info), 0, 3, 32, 0) == -1   # panel 0
    assert lib.mp_lu_ex(4, 200, fake, 4, 16, fake, ctypes.byref(info), 64, 3, 32, 0) == -2


def test_batched_alias_across_items_without_device(mp):
    """A result of one item overlapping an operand or result of another item is
    rejected (all leaves of a batch run in one launch); disjoint buffers and
    operands shared between items pass validation (the call then needs the
    device, which a CPU host does not have: MP_E_DEVICE or MP_OK, never
    MP_E_ALIAS)."""
    lib = mp.lib
    L = 256 // 32
    words = (L + 2) * 16            # one 4 x 4 matrix

    def batch(ptrs):
        cnt = len(ptrs)
        i64 = ctypes.c_int64 * cnt
        vp = ctypes.c_void_p * cnt
        four = i64(*([4] * cnt))
        sixteen = i64(*([16] * cnt))
        A = vp(*[ctypes.c_void_p(a) for a, _, _ in ptrs])
        B = vp(*[ctypes.c_void_p(b) for _, b, _ in ptrs])
        C = vp(*[ctypes.c_void_p(c) for _, _, c in ptrs])
        return lib.mp_gemm_batched(cnt, four, four, four, 256, 0, 0, A, four, sixteen, B, four, sixteen,
                                   C, four, sixteen)

    base = 1 << 40
    at = lambda k: base + 4 * words * k
    # item 1's result is item 0's A
    assert batch([(at(0), at(1), at(2)), (at(3), at(4), at(0))]) == -3
    # item 0's result overlaps item 1's B by one word
    assert batch([(at(0), at(1), at(2)), (at(3), at(2) + 4 * words - 4, at(5))]) == -3
    # two results overlap
    assert batch([(at(0), at(1), at(2)), (at(3), at(4), at(2) + 4)]) == -3
    # shared operands, disjoint results: not an alias error
    assert batch([(at(0), at(1), at(2)), (at(0), at(1), at(3))]) != -3


def test_slice_inner_size_limit_without_device(mp):
    lib = mp.lib
    l = 131009
    base = 1 << 40
    L = 256 // 32
    A = base
    B = base + 4 * (L + 2) * 4 * l + (1 << 20)
    C = B + 4 * (L + 2) * 4 * l + (1 << 20)
    w = (ctypes.c_int * 2)()
    rc = lib.mp_gemm_slice(4, l, 4, 256, 64, ctypes.c_void_p(A), l, 4 * l, ctypes.c_void_p(B), 4, 4 * l,
                           ctypes.c_void_p(C), 4, 16, w)
    assert rc == -6, rc
    assert "131008" in mp.last_error()


def test_launch_settings_without_device(mp):
    lib = mp.lib
    assert lib.mp_set_launch(3, 0) == -1
    assert lib.mp_set_launch(7, 0) == -1
    assert lib.mp_set_launch(0, 2) == -1
    assert lib.mp_set_launch(5, 1) == 0
    assert lib.mp_set_launch(0, 0) == 0
