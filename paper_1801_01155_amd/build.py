"""Builds liblineset.so (HIP, gfx950) next to this file.

    python -m paper_1801_01155_amd.build

Every HIP source under csrc/ is compiled by hipcc into one shared library
with a C ABI (include/lineset.h). Floating-point contraction is off so that
the fp64 ray set-up, grid walk and lattice snapping round exactly as
documented; packed fp32 instructions are disabled.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblineset.so")
ARCH = os.environ.get("LINESET_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, extra=None) -> str:
    out_tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *(extra or []), "-o", out_tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
