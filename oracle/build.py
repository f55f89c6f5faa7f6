"""Build the CPU oracle library (test infrastructure) with gcc.

The oracle is compiled without FMA contraction and without fast-math, so each
arithmetic operation is one correctly rounded IEEE double operation.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpco.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB,
           os.path.join(HERE, "pco.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


def ensure() -> str:
    src = os.path.join(HERE, "pco.c")
    hdr = os.path.join(HERE, "pco.h")
    if (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(src)
            or os.path.getmtime(LIB) < os.path.getmtime(hdr)):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
