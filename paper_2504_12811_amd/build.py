"""Build the gfx950 HIP library (libaaa_hip.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaaa_hip.so")
SOURCES = ["api.hip", "preprocess.hip", "emit.hip", "sort.hip", "blend.hip", "backward.hip", "train_freq.hip", "adam.hip",
           "peaks.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions are disabled throughout
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # native float atomic adds (device memory is coarse-grained)
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    # every symbol resolved at link time (a missing definition fails the build)
    "-Wl,-z,defs",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.exists(c) or c == "hipcc"):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include")] + (extra or []) + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
