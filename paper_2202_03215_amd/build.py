"""Compile the gfx950 HIP library (libpc.so) in-tree with hipcc.

Flags: no FMA contraction (every product and sum rounded separately, so the
particle arithmetic is reproducible), no packed-FP32 instructions, -O3, and
no compiler rewriting of atomics into wave-level aggregates (the kernels
aggregate their atomics themselves, mostly from one lane; the rewrite added
a third of the electron push's instructions).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpc.so")
SOURCES = ["csrc/kernels.hip", "csrc/api.hip", "csrc/mlp.hip", "csrc/fluid.hip"]
DEPS = SOURCES + ["csrc/device.h", "csrc/launch.h"]


def hipcc() -> str:
    for p in (os.environ.get("HIPCC", ""), "/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if p and os.path.exists(p):
            return p
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
           "-I", os.path.join(ROOT, "include"), "-o", tmp]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    inc = os.path.join(HERE, "..", "include")
    deps = DEPS + [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return any(os.path.getmtime(os.path.join(HERE, d)) > t for d in deps)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
