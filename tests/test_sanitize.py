"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/sanitize/host_driver (the library's host sources built with both
sanitizers on the host side, kernels from libpond.so) driven through the C
ABI.  The CPU test builds the driver and runs its host-only scenario; the
GPU test runs the device scenario with the driver the CPU test built."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "sanitize", "_build", "host_driver")
SOURCES = [os.path.join(HERE, "sanitize", "host_driver.cpp")] + [
    os.path.join(HERE, "..", "paper_1503_01405_amd", "csrc", f)
    for f in ("pond_api.cpp", "pond_search.cpp", "pond_serve.cpp", "pond_aid.cpp", "pond_static.cpp",
              "pond_tune.cpp", "pond_internal.hpp", "pond_tune.hpp")] + [
    os.path.join(HERE, "..", "include", "pond.h")]
SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(mode, timeout):
    env = dict(os.environ, **SAN_ENV)
    r = subprocess.run([DRIVER, mode], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert r.returncode == 0, r.returncode
    assert f"driver {mode}: 0 failed checks" in r.stdout


@pytest.mark.skipif(shutil.which(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")) is None,
                    reason="hipcc not installed")
def test_host_runtime_sanitized_cpu_scenario():
    subprocess.run([sys.executable, os.path.join(HERE, "sanitize", "build_driver.py")], check=True,
                   capture_output=True, timeout=600)
    _run("cpu", 120)


@pytest.mark.gpu
def test_host_runtime_sanitized_gpu_scenario():
    if not os.path.exists(DRIVER):
        pytest.skip("sanitizer driver not built (the CPU test builds it)")
    if max(os.path.getmtime(s) for s in SOURCES) > os.path.getmtime(DRIVER):
        pytest.skip("sanitizer driver older than its sources (the CPU test rebuilds it)")
    print("case: sanitized host runtime, device scenario", flush=True)
    _run("gpu", 240)
