"""Build libpond.so (HIP kernels + C ABI) for gfx950, in-tree.

Usage: python paper_1503_01405_amd/build.py  (runs without importing the
package, whose import loads the library this script builds).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpond.so")

SOURCES = ["pond_kernels.hip", "pond_api.cpp", "pond_search.cpp", "pond_serve.cpp", "pond_aid.cpp"]
HEADERS = ["pond_fft.hpp", "pond_internal.hpp"]

# -ffp-contract=off: no implicit fused multiply-adds, so the float64 fold
# phase and plan geometry round exactly as written (fmaf is used explicitly
# where a fused operation is wanted).  Packed fp32 instructions are turned
# off for the device code.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source into libpond.so next to this file; returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for s in SOURCES:
        if s.endswith(".cpp"):
            cmd += ["-x", "hip", os.path.join(CSRC, s)]
        else:
            cmd += [os.path.join(CSRC, s)]
    cmd += ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpond.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
