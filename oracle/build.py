"""Build the CPU oracle library (test infrastructure) with gcc.

The oracle is compiled without FMA contraction and without fast-math, so each
arithmetic operation is one correctly rounded IEEE double operation.  Two
builds of the same source: libpco.so (serial, the parity reference) and
libpco_omp.so (-fopenmp, the all-core timing build; it computes bit for bit
what the serial build computes).  A third build, libpco_asan.so
(-fsanitize=address,undefined, host code only), is what the sanitizer test
loads when PCO_SANITIZE=1 is set.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpco.so")
LIB_OMP = os.path.join(HERE, "libpco_omp.so")
LIB_ASAN = os.path.join(HERE, "libpco_asan.so")


def sanitized() -> bool:
    return os.environ.get("PCO_SANITIZE", "") == "1"


def _path(omp: bool) -> str:
    if sanitized():
        return LIB_ASAN
    return LIB_OMP if omp else LIB


def build_one(omp: bool, verbose: bool = False) -> str:
    out = _path(omp)
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-shared", "-fPIC"]
    if sanitized():
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas"]
    else:
        cmd += ["-fopenmp"] if omp else ["-Wno-unknown-pragmas"]
    cmd += ["-o", out, os.path.join(HERE, "pco.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def build(verbose: bool = False) -> str:
    build_one(True, verbose)
    return build_one(False, verbose)


def ensure(omp: bool = False) -> str:
    lib = _path(omp)
    src = os.path.join(HERE, "pco.c")
    hdr = os.path.join(HERE, "pco.h")
    if (not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src)
            or os.path.getmtime(lib) < os.path.getmtime(hdr)):
        build_one(omp)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
