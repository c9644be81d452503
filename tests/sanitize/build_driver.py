"""Builds tests/sanitize/host_driver: the library's host sources and the
driver compiled with AddressSanitizer and UndefinedBehaviorSanitizer on the
host side only (device code is never sanitized), linked against the normal
libpond.so for the kernels and their launchers.  Output:
tests/sanitize/_build/host_driver.  Usage: python tests/sanitize/build_driver.py"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1503_01405_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_1503_01405_amd")
OUT = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HOST_SOURCES = ["pond_api.cpp", "pond_search.cpp", "pond_serve.cpp", "pond_aid.cpp", "pond_static.cpp",
                "pond_tune.cpp"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-x", "hip",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build():
    os.makedirs(OUT, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES] + [os.path.join(HERE, "host_driver.cpp")]
    objs = [os.path.join(OUT, os.path.basename(s) + ".o") for s in srcs]

    def cc(so):
        s, o = so
        return subprocess.run([hipcc, *FLAGS, *SAN, "-c", s, "-o", o], capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=7) as ex:
        res = list(ex.map(cc, zip(srcs, objs)))
    for s, r in zip(srcs, res):
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise SystemExit(f"compile failed: {s}")
    exe = os.path.join(OUT, "host_driver")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    link = [clang, "-fsanitize=address,undefined", "-g", *objs, "-L", LIBDIR, "-lpond",
            f"-Wl,-rpath,{LIBDIR}", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
            f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise SystemExit("link failed")
    return exe


if __name__ == "__main__":
    print(build())
