"""Build the C oracle (oracle/c/mpref.c) into oracle/c/libmpref.so with gcc.

Test infrastructure: called by the tests, __graft_entry__.build() and the
benchmark's CPU-baseline leg.  Plain gcc -O2 with OpenMP; nothing tuned.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpref.c")
LIB = os.path.join(HERE, "libmpref.so")


def build(force=False):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
