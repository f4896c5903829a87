"""Build the HIP library for gfx950 (in-tree): paper_1607_02214_amd/libppmlr.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libppmlr.so")
SOURCES = [os.path.join(CSRC, "ppmlr_lib.hip")]
HEADERS = [os.path.join(CSRC, "ppmlr_sweep.hpp"), os.path.join(ROOT, "include", "ppmlr.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # multiply-adds are fused only where the source writes them in one
    # expression, so every instantiation of the sweep (single run, ensemble,
    # with or without counters) rounds identically
    "-ffp-contract=on",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + (extra or []) + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
