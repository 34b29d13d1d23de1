"""Builds the C part of the oracle (liboracle.so) with gcc.

Test infrastructure only.  Run as ``python -m oracle.build`` or through
``__graft_entry__.build()``.  Building the checker does not use it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["exact.c", "dd.c"]


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", LIB] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


def ensure_built():
    if not os.path.exists(LIB):
        return build()
    newest = max(os.path.getmtime(os.path.join(HERE, s)) for s in SOURCES)
    if os.path.getmtime(LIB) < newest:
        return build()
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
