"""Build libpond.so (HIP kernels + C ABI) for gfx950, in-tree.

Every source is compiled to an object of its own, in parallel, then linked.

Usage: python paper_1503_01405_amd/build.py  (runs without importing the
package, whose import loads the library this script builds).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpond.so")

KERNEL_SOURCES = ["pond_k1.hip", "pond_k2.hip", "pond_k3.hip", "pond_fold.hip", "pond_real.hip",
                  "pond_aid_kernels.hip", "pond_split.hip"]
HOST_SOURCES = ["pond_api.cpp", "pond_search.cpp", "pond_serve.cpp", "pond_aid.cpp", "pond_static.cpp",
                "pond_tune.cpp"]
SOURCES = KERNEL_SOURCES + HOST_SOURCES
HEADERS = ["pond_fft.hpp", "pond_device.hpp", "pond_internal.hpp", "pond_tune.hpp"]

# -ffp-contract=off: no implicit fused multiply-adds, so the float64 fold
# phase and plan geometry round exactly as written (fmaf is used explicitly
# where a fused operation is wanted).  Packed fp32 instructions are turned
# off for the device code.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str, extra: list[str]) -> tuple[str, subprocess.CompletedProcess]:
    cmd = [hipcc()] + FLAGS + extra + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c"]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += [os.path.join(CSRC, src), "-o", obj]
    return src, subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, out: str = LIB, extra: list[str] | None = None, jobs: int = 8) -> str:
    """Compile every source into `out` (default libpond.so next to this
    file); `extra` flags go to every compile and the link.  Returns the path."""
    extra = list(extra or [])
    tmpdir = tempfile.mkdtemp(prefix="pond_build_")
    try:
        objs = [os.path.join(tmpdir, s + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
            results = list(ex.map(lambda so: _compile(so[0], so[1], extra), zip(SOURCES, objs)))
        failed = False
        for src, res in results:
            if res.returncode != 0:
                failed = True
                sys.stderr.write(f"---- {src}\n" + res.stdout + res.stderr)
            elif verbose:
                sys.stderr.write(res.stderr)
        if failed:
            raise RuntimeError("hipcc failed building libpond.so")
        tmp = out + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + extra + objs + ["-o", tmp]
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libpond.so")
        os.replace(tmp, out)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
