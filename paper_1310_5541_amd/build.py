"""Compile the gfx950 HIP library ``libpcsir.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpcsir.so")
SOURCES = [os.path.join(CSRC, "pcsir.hip"), os.path.join(CSRC, "mlp.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("kernels.h", "device_util.h", "mlp_device.h", "surrogate.h")] + [
    os.path.join(os.path.dirname(HERE), "include", h) for h in ("pcsir.h", "pcsir_mlp.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add fusion: the compensated (TwoSum / TwoProduct)
    # sums rely on each operation rounding where it is written; fused
    # multiply-adds are written explicitly (fmaf) where they are wanted
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpcsir.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
