"""Builds libcafgpu.so (the compute-actor C ABI) for gfx950 with hipcc.

Flags that matter for correctness:
  -ffp-contract=off   no fused multiply-add: escape-time counts must equal
                      the CPU reference's bit for bit;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keeps the compiler from emitting packed fp32 math.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcafgpu.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "runtime.cpp", "drive.cpp",
                                                  "offload.cpp")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("caf_internal.h", "tiles.h")] + [
    os.path.join(ROOT, "include", "caf_gpu.h")]
ARCH = os.environ.get("CAFGPU_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-ffp-contract=off", "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, extra=()) -> str:
    cmd = ["hipcc", *FLAGS, *extra, "-o", LIB + ".tmp", *SOURCES, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
