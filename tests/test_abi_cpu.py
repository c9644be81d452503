"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/pond.h declares, and rejects invalid plans before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pond.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pond_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_path_calls():
    names = _declared()
    for n in ("pond_plan_create", "pond_dedisperse_fold", "pond_dedisperse_series", "pond_plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1503_01405_amd.pond as B
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) <= set(B.EXPORTS)


@pytest.mark.parametrize("args", [
    (326.5, 16.0, 1.0, (1 << 18) + 1, 256, 0.0891),   # nfft not a power of two
    (326.5, 16.0, 1.0, 1 << 9, 256, 0.0891),          # nfft below 2^10
    (326.5, 16.0, 1.0, 1 << 28, 256, 0.0891),         # nfft above 2^27
    (326.5, 16.0, -1.0, 1 << 18, 256, 0.0891),        # negative DM
    (326.5, 16.0, float("nan"), 1 << 18, 256, 0.0891),
    (326.5, 0.0, 1.0, 1 << 18, 256, 0.0891),          # zero bandwidth
    (5.0, 16.0, 1.0, 1 << 18, 256, 0.0891),           # band edge below 0 MHz
    (326.5, 16.0, 1.0, 1 << 18, 0, 0.0891),           # no bins
    (326.5, 16.0, 1.0, 1 << 18, 65537, 0.0891),       # too many bins
    (326.5, 16.0, 1.0, 1 << 18, 256, 0.0),            # period
    (326.5, 16.0, 1.0, 1 << 18, 256, 1e-9),           # period shorter than a sample
    (326.5, 16.0, 200.0, 1 << 20, 256, 0.0891),       # smear longer than the FFT
])
def test_invalid_plans_are_rejected_before_device_work(args):
    import paper_1503_01405_amd as P
    with pytest.raises(P.PondError) as ei:
        P.pond_plan_create(*args)
    assert ei.value.code == P.POND_EINVAL


def test_null_plan_calls():
    import paper_1503_01405_amd.pond as B
    lib = B.lib()
    assert lib.pond_dedisperse_fold(None, None, 0, 0, None, 0, None) == B.POND_EINVAL
    assert lib.pond_plan_query(None, None) == B.POND_EINVAL
    assert lib.pond_plan_expect(None, 0, 0, None, None) == B.POND_EINVAL
    lib.pond_plan_destroy(None)
    assert lib.pond_strerror(B.POND_EDEVICE)
    assert lib.pond_real_dedisperse(None, None, 0, 0, None, 0, 32, None, 0, None, None) == B.POND_EINVAL
    assert lib.pond_real_expect(None, 0, 0, None, None) == B.POND_EINVAL
    assert lib.pond_aid_run(None, None, 0, None, None, 0, None) == B.POND_EINVAL


def test_copy_arguments_are_checked_before_device_work():
    import paper_1503_01405_amd.pond as B
    lib = B.lib()
    assert lib.pond_copy_device(None, None, 0, None) == B.POND_OK          # nothing to copy
    assert lib.pond_copy_device(None, None, 16, None) == B.POND_EINVAL      # null pointers
    assert lib.pond_copy_device(4096, 8192, 15, None) == B.POND_EINVAL      # not whole 16-byte words
    assert lib.pond_copy_device(4104, 8192, 16, None) == B.POND_EINVAL      # misaligned destination
    assert lib.pond_copy_device(4096, 8200, 16, None) == B.POND_EINVAL      # misaligned source
    assert lib.pond_copy_device(4096, 8192, -16, None) == B.POND_EINVAL


@pytest.mark.parametrize("args", [
    (326.5, 16.0, 1.0, 1 << 20, 256, 0.0891, 0, 0, 5),           # no such sideband
    (326.5, 16.0, 1.0, (1 << 20) + 2, 256, 0.0891, 0, 0, 0),     # real block not a power of two
    (326.5, 16.0, 1.0, 1 << 10, 256, 0.0891, 0, 0, 0),           # packed length below 2^10
    (326.5, 16.0, 1.0, 1 << 20, 256, 0.0891, 1, 0, 1),           # matrix-core form not offered
    (326.5, 16.0, 1.0, 1 << 20, 256, 0.0891, 3, 0, 1),           # packed float16 form not offered
    (326.5, 16.0, 200.0, 1 << 21, 256, 0.0891, 0, 0, 0),         # smear longer than the block
])
def test_invalid_real_plans_are_rejected_before_device_work(args):
    import paper_1503_01405_amd.pond as B
    lib = B.lib()
    assert not lib.pond_real_plan_create(*args)
    assert lib.pond_create_status() == B.POND_EINVAL


def test_library_shares_torchs_hip_runtime():
    """The binding loads torch before libpond.so, so the library's HIP
    runtime dependency resolves to the copy torch already loaded (a second
    runtime in the process would not see torch's device state)."""
    import subprocess
    import sys
    code = ("import paper_1503_01405_amd, torch, os\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "paths = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
            "print(len(paths)); print(paths)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.splitlines()[0] == "1", out.stdout


@pytest.mark.parametrize("dm,nfft", [(0.0, 1 << 10), (0.003, 1 << 10), (1.0, 1 << 18), (50.0, 1 << 23),
                                     (130.0, 1 << 24), (200.0, 1 << 24), (200.0, 1 << 23), (37.2, 1 << 20)])
def test_library_geometry_equals_the_oracle_rule(dm, nfft):
    """pond_geometry (host arithmetic of the plan) against the oracle's
    geometry of the same block: identical n_front, discard and hop, and
    both refuse a block shorter than the smear."""
    import oracle as O
    import paper_1503_01405_amd.pond as B
    got = B.pond_geometry(326.5, 16.0, dm, nfft)
    try:
        g = O.plan_geometry(326.5, 16.0, dm, nfft)
        want = (g["n_front"], g["discard"], g["hop"])
    except ValueError:
        want = None
    assert got == want


def test_library_geometry_rejects_bad_arguments():
    import paper_1503_01405_amd.pond as B
    assert B.pond_geometry(326.5, 16.0, 1.0, 3000) is None
    assert B.pond_geometry(326.5, -1.0, 1.0, 1 << 18) is None
    assert B.pond_geometry(326.5, 16.0, -0.5, 1 << 18) is None
