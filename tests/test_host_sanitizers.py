"""Host code under the address and undefined-behaviour sanitizers (CPU only).

* The library's planner (paper_1410_1599_amd/csrc/plan.cpp, host C++ with no
  device code), built with g++ -fsanitize=address,undefined together with a
  small driver (tests/host/plan_driver.cpp), plans thousands of products and
  batches; every plan must pass its own bounds validation, its operation
  counts and depth must equal the Python oracle's, and the sanitizers must
  report nothing (any finding aborts the driver).
* The C oracle (oracle/c/mpref.c), narrow and wide builds instrumented the
  same way, runs products of every algorithm and odd-size policy, LU with and
  without pivoting, the solve, the residual and scalar operations in a child
  process that preloads the sanitizer runtime, and must agree with the
  Python oracle.
"""

import itertools
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

from oracle import gemm as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_1599_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

needs_gxx = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no g++/gcc")


def sanitizer_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def plan_driver():
    d = tempfile.mkdtemp(prefix="plan_san_")
    exe = os.path.join(d, "plan_driver")
    cmd = ["g++", "-std=c++17"] + SAN + ["-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-I" + CSRC,
                                         os.path.join(CSRC, "plan.cpp"),
                                         os.path.join(ROOT, "tests", "host", "plan_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("planner does not build with g++ here: " + r.stderr[-500:])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def run_driver(exe, lines):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    return [tuple(float(v) for v in line.split()) for line in r.stdout.splitlines()]


@needs_gxx
def test_planner_under_sanitizers_matches_oracle_counts(plan_driver):
    dims = [1, 3, 8, 31, 33, 65, 100]
    cases, lines = [], []
    pol = {"peel": 0, "pad": 1, "mixed": 2}
    for (m, l, n), algo, cut, policy in itertools.product(itertools.product(dims, repeat=3), ("strassen", "winograd"),
                                                          (4, 32), ("peel", "pad", "mixed")):
        cases.append((m, l, n, algo, cut, policy))
        lines.append("%d %d %d 8 %d %d %d 0 0" % (m, l, n, 2 if algo == "strassen" else 3, cut, pol[policy]))
    for (m, l, n), L, leaf, tcl in itertools.product(((300, 200, 100), (1, 1, 1), (257, 64, 33)), (4, 8, 32, 64),
                                                     (0, 1), (0, 4, 5)):
        cases.append((m, l, n, "simple", 0, "peel"))
        lines.append("%d %d %d %d %d 0 0 %d %d" % (m, l, n, L, leaf, leaf, tcl))
    out = run_driver(plan_driver, lines)
    assert len(out) == len(cases)
    for (m, l, n, algo, cut, policy), (depth, nmul, nadd, ws, nl, nleaf, valid) in zip(cases, out):
        assert valid == 1, (m, l, n, algo, cut, policy)
        assert (nmul, nadd) == G.op_counts(m, l, n, algo, max(cut, 1), policy), (m, l, n, algo, cut, policy)
        if algo != "simple":
            assert depth == G.depth(m, l, n, cut, policy)


@needs_gxx
def test_batched_planner_under_sanitizers(plan_driver):
    lines = ["batch 3", "100 80 90 8 3 16 0 0 0", "33 1 7 8 3 16 0 0 0", "65 65 65 8 3 16 0 0 0",
             "batch 2", "1 1 1 4 2 4 2 0 5", "200 3 150 4 2 4 2 0 5",
             "batch 1", "129 130 131 64 3 32 1 0 0"]
    out = run_driver(plan_driver, lines)
    assert len(out) == 3 and all(o[-1] == 1 for o in out)
    want = [sum(G.op_counts(m, l, n, "winograd", 16, "peel")[0] for m, l, n in ((100, 80, 90), (33, 1, 7), (65, 65, 65)))]
    assert out[0][1] == want[0]


CHILD = r'''
import os, random, sys
sys.path.insert(0, %(root)r)
sys.path.insert(0, os.path.join(%(root)r, "tests"))
from helpers import adversarial_pairs
from oracle import cref, gemm as G, lu as LU, mpnum
from paper_1410_1599_amd import inputs as I
for p in (128, 256, 1024, 2048):
    A = I.uniform_pm1(7, 6, p, 1); B = I.log_uniform(6, 9, p, 2, -5, 5)
    Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
    for algo in ("simple", "block", "strassen", "winograd"):
        for policy in ("peel", "pad", "mixed"):
            got = I.from_planes(cref.gemm(A, B, p, algo=algo, cutoff=1, policy=policy, block_size=4), p)
            assert got == G.gemm(Ao, Bo, p, algo=algo, cutoff=1, policy=policy, block_size=4), (p, algo, policy)
    for pivot in (True, False):
        M = I.uniform_pm1(9, 9, p, 3) if pivot else I.lotkin(9, p)
        F, piv, info = cref.lu(M, p, panel=4, algo="winograd", cutoff=1, pivot=pivot)
        Fp, pivp, infop = LU.lu(I.from_planes(M, p), p, panel=4, algo="winograd", cutoff=1, pivot=pivot)
        assert I.from_planes(F, p) == Fp and list(piv) == pivp
        b = cref.gemm(M, I.ones_column(9, p), p, algo="simple")
        cref.lu_solve(F, piv, b, p)
        cref.lu_residual(M, F, piv, p)
    rng = random.Random(p)
    def rec(v):
        a = I.empty(1, 1, p); I.set_entry(a, 0, 0, v, p); return a.reshape(-1).copy()
    for x, y in rng.sample(adversarial_pairs(rng, p), 60):
        for op, f in (("mul", mpnum.mul), ("add", mpnum.add), ("sub", mpnum.sub), ("div", mpnum.div)):
            if op == "div" and y[0] == 0:
                continue
            r = cref.scalar(op, p, rec(x), rec(y))
            assert I.entry(r.reshape(p // 32 + 2, 1, 1), 0, 0, p) == f(x, y, p), (op, p)
print("child ok")
'''


@needs_gxx
def test_c_oracle_under_sanitizers():
    rt = sanitizer_runtime()
    if rt is None:
        pytest.skip("no libasan runtime")
    from oracle.c import build as cbuild
    cbuild.build(sanitize=True)
    cbuild.build(wide=True, sanitize=True)
    env = dict(os.environ, MPREF_SANITIZE="1", LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT}], capture_output=True, text=True, env=env,
                       timeout=900)
    assert r.returncode == 0 and "child ok" in r.stdout, (r.stdout[-1000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
