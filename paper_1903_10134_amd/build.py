"""Build the gfx950 HIP library ``libmdpd.so`` in-tree with hipcc.

Flags:
  --offload-arch=gfx950                        MI355X (CDNA4) only
  -ffp-contract=on                             fuse a*b+c only inside one expression,
                                               and honour "fp contract(off)" scopes
                                               (the exact neighbour test relies on it)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                               no packed FP32 instructions
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmdpd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def asm(source: str, out: str) -> None:
    """Write the gfx950 assembly of one source file (for inspection)."""
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")], "--cuda-device-only", "-S",
           os.path.join(CSRC, source), "-o", out]
    subprocess.check_call(cmd)


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
