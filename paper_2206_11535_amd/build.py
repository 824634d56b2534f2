"""Build the HIP library (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "mu3e.hip")
LIB = os.path.join(PKG, "libmu3e.so")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-mcode-object-version=5",
    # no packed float32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # float32 division and square root by the hardware reciprocal / root
    # (within 2 ulp) instead of the correctly rounded sequences: the float32
    # paths decide nothing within a few ulp of an edge (their margins are
    # orders of magnitude wider), and the track fit is bound by these sequences
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-Wall",
]


def build(verbose: bool = False) -> str:
    """Compile libmu3e.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
