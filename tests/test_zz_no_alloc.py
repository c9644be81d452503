"""The no-allocation entry point (pond_dedisperse_segment_noalloc) against
the plan path it mirrors (pond_plan_create_ex + pond_dedisperse_series +
the end-of-stream call, one open-ended sub-integration), through the C ABI:
two calls in a row on one device, the second with a smaller input (the
shared static scratch keeps the first call's contents, which must not leak
into the second).  Same kernels and tables, integer fold: the profile and
the series are expected bit for bit, and asserted within the float32
tolerance of the parity tests (profile 1e-6, series 1e-5) in any case."""
import numpy as np
import pytest

import synth
from gpu_helpers import BW, F0, rel_l2

pytestmark = pytest.mark.gpu


def _plan_path(P, iq_dev, nsamp, dm, nfft, nbins, period, prec, decim):
    import torch
    h = P.pond_plan_create(F0, BW, dm, nfft, nbins, period, prec)
    try:
        nprof, nout = P.pond_plan_expect(h, nsamp, 0)
        ser = torch.empty(max(1, nout // decim), device="cuda")
        prof = torch.zeros((1, nbins), device="cuda")
        r, n = P.pond_dedisperse_series(h, iq_dev, nsamp, 0, prof, 0, decim, ser, ser.numel())
        assert r == 0 and n == nout // decim
        assert P.pond_dedisperse_fold(h, None, 0, 0, prof, 1) == (1 if nout else 0)
        torch.cuda.synchronize()
        return prof[0].cpu().numpy(), ser[:n].cpu().numpy()
    finally:
        P.pond_plan_destroy(h)


def _noalloc(P, iq_dev, nsamp, dm, nfft, nbins, period, prec, decim, cap):
    import torch
    prof = torch.full((nbins,), -1.0, device="cuda")
    ser = torch.full((max(1, cap),), -1.0, device="cuda")
    n = P.pond_dedisperse_segment_noalloc(F0, BW, dm, nfft, nbins, period, prec, iq_dev, nsamp, decim, prof,
                                          ser, cap)
    torch.cuda.synchronize()
    assert n >= 0, n
    return prof.cpu().numpy(), ser[:n].cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "mixed_valu"])
def test_noalloc_matches_plan_path_twice(precision):
    import torch
    import paper_1503_01405_amd as P
    prec = P.FORMS[precision]
    # first call: 2^20 blocks at DM 5, 1024 bins; second: smaller input,
    # 2^16 blocks at DM 0.7, 300 bins, decim 4
    cases = [(5.0, 1 << 20, 1024, 0.0891, 16, 9_000_007), (0.7, 1 << 16, 300, 4.1e-3, 4, 1_500_003)]
    for k, (dm, nfft, nbins, period, decim, nsamp) in enumerate(cases):
        print(f"case: no-alloc {precision} call {k} dm={dm} nfft=2^{nfft.bit_length() - 1} nsamp={nsamp}",
              flush=True)
        iq = torch.from_numpy(synth.white_stream_int8(90 + k, nsamp)).to("cuda")
        want_p, want_s = _plan_path(P, iq, nsamp, dm, nfft, nbins, period, prec, decim)
        got_p, got_s = _noalloc(P, iq, nsamp, dm, nfft, nbins, period, prec, decim, want_s.size)
        assert got_s.size == want_s.size
        ep, es = rel_l2(got_p, want_p), rel_l2(got_s, want_s)
        print(f"{precision} call {k}: profile rel-L2 {ep:.2e} series rel-L2 {es:.2e} "
              f"bitwise {np.array_equal(got_p, want_p) and np.array_equal(got_s, want_s)}", flush=True)
        assert ep <= 1e-6 and es <= 1e-5


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    import paper_1503_01405_amd as P
    iq = torch.zeros(2 * 4096, dtype=torch.int8, device="cuda")
    prof = torch.zeros(16, device="cuda")
    ser = torch.zeros(1024, device="cuda")
    f = P.pond_dedisperse_segment_noalloc
    assert f(F0, BW, 0.01, 1 << 21, 16, 0.01, P.POND_FP32, iq, 4096, 16, prof, ser, 1024) == P.POND_EINVAL
    assert f(F0, BW, 0.01, 1 << 12, 8193, 0.01, P.POND_FP32, iq, 4096, 16, prof, ser, 1024) == P.POND_EINVAL
    assert f(F0, BW, 0.01, 1 << 12, 16, 0.01, P.POND_HALF, iq, 4096, 16, prof, ser, 1024) == P.POND_EINVAL
    assert f(F0, BW, 0.01, 1 << 12, 16, 0.01, P.POND_FP32, iq, 4096, 16, prof, ser, 0) == P.POND_EINVAL
    hop = P.pond_geometry(F0, BW, 0.01, 1 << 12)[2]
    assert f(F0, BW, 0.01, 1 << 12, 16, 0.01, P.POND_FP32, iq, 4096, 16, prof, ser, 1024) == hop // 16
    torch.cuda.synchronize()
