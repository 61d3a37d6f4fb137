"""Build the C oracle (oracle/c/mpref.c) with gcc into two libraries:

* libmpref.so: values up to 48 limbs (1536 bits; the LU residual runs at
  2p + 64 bits, so 512-bit LU residuals fit);
* libmpref_wide.so: the same source with up to 656 limbs (10240-bit values
  and their 2p + 64-bit residuals).  Larger fixed records make it slower, so
  the narrow build serves every precision it can hold.

Test infrastructure: called by the tests, __graft_entry__.build() and the
benchmark's CPU-baseline leg.  Plain gcc -O2 with OpenMP; nothing tuned.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpref.c")
LIB = os.path.join(HERE, "libmpref.so")
LIB_WIDE = os.path.join(HERE, "libmpref_wide.so")
MAXL_WIDE = 656


# the host sanitizer builds (tests/test_host_sanitizers.py): address and
# undefined-behaviour checks, every finding fatal
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _build_one(lib, defines, force):
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= max(os.path.getmtime(SRC),
                                                                           os.path.getmtime(__file__)):
        return lib
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall"] + defines + ["-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(force=False, wide=False, sanitize=False):
    """Path of the narrow library (wide=False) or of the wide one; sanitize
    gives the address / undefined-behaviour instrumented twin of either."""
    lib, defines = (LIB_WIDE, ["-DMAXL=%d" % MAXL_WIDE]) if wide else (LIB, [])
    if sanitize:
        lib = lib.replace(".so", "_san.so")
        defines = defines + SANITIZE
    return _build_one(lib, defines, force)


def build_all(force=False):
    return build(force), build(force, wide=True)


if __name__ == "__main__":
    print(build_all(force="--force" in sys.argv))
