"""Build libmpgemm.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Every source under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_1410_1599_amd/libmpgemm.so.  Runs on a machine without
a GPU: hipcc cross-compiles the device code.

    python -m paper_1410_1599_amd.build [--force]
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmpgemm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# no packed FP32 instructions: the kernels are integer code, and the packed
# forms are kept out of every HIP object
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(os.path.dirname(HERE), "include")]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def headers():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(os.path.dirname(HERE), "include", "mpgemm.h"))
    return hs


# the product at 1024 bits is a fully unrolled 32 x 32-limb column loop; under
# the default threshold the compiler leaves it rolled and indexes the limbs
# through a stack array (scratch memory)
UNROLL = ["-mllvm", "-pragma-unroll-threshold=500000"]
EXTRA_FLAGS = {"gemm_kernels.hip": UNROLL, "lu_kernels.hip": UNROLL}


def _compile(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [HIPCC] + HIP_FLAGS + EXTRA_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + HIP_FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, msgs))
    return obj, msgs


def build(force=True, jobs=None, verbose=False):
    """Compile every source and link the library; returns its path."""
    os.makedirs(OUT, exist_ok=True)
    srcs = sources()
    newest_input = max(os.path.getmtime(p) for p in srcs + headers() + [__file__])
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= newest_input:
        return LIB
    jobs = jobs or min(8, len(srcs))
    newest_header = max(os.path.getmtime(p) for p in headers() + [__file__])

    def fresh(src):                     # incremental builds reuse objects newer than every input
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        return (not force and os.path.exists(obj)
                and os.path.getmtime(obj) >= max(os.path.getmtime(src), newest_header))

    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda src: (os.path.join(OUT, os.path.basename(src) + ".o"), "") if fresh(src)
                              else _compile(src), srcs))
    for _, msgs in results:
        if verbose and msgs.strip():
            print(msgs)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose="-v" in sys.argv))
