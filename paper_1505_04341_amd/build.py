"""Builds libddlr.so (HIP for gfx950 + host setup) in the package directory."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libddlr.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("ddlr_api.hip", "host_setup.cpp", "partition.cpp", "cinv.cpp", "cheb.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code (some forms have
# produced silently wrong results on this hardware class).
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def command(out: str = LIB) -> list[str]:
    return [HIPCC, "-O3", "-std=c++17", "-fPIC", "-shared", *DEVICE_FLAGS, "-I", os.path.join(ROOT, "include"),
            "-I", os.path.join(HERE, "csrc"), "-Wall", "-Wno-unused-function", "-o", out, *SOURCES]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
