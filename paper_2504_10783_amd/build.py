"""Builds the HIP library `libezo.so` in-tree for gfx950 with hipcc.

    python -m paper_2504_10783_amd.build

Packed FP32 instructions are disabled for the whole device compile
(`-target-feature -packed-fp32-ops`); hipcc's host pass warns that it does
not know the feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", f) for f in ("ezo_api.hip", "ezo_surrogate.hip", "ezo_tune.hip")]
OUT = os.path.join(PKG, "libezo.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
