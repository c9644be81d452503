"""A whole call sequence (append a stream, end it) captured into a HIP graph
and replayed gives the eager results, replay after replay, with eager work
and synchronisation in between."""
import numpy as np
import pytest

import synth
from gpu_helpers import BW, F0

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_valu", "half"])
def test_graph_replay_matches_eager(precision):
    import torch
    import paper_1503_01405_amd as P

    nfft, dm, nbins, period, subint, decim = 1 << 18, 1.0, 256, synth.PERIOD_S, 1_000_000, 16
    nsamp = 3_000_001
    print(f"case: graph replay {precision} nfft=2^18 nsamp={nsamp}", flush=True)
    x = torch.from_numpy(synth.white_stream_int8(21, nsamp)).to("cuda")
    h = P.pond_plan_create(F0, BW, dm, nfft, nbins, period, P.FORMS[precision])
    try:
        nprof, nout = P.pond_plan_expect(h, nsamp, subint)
        prof = torch.zeros((nprof + 1, nbins), device="cuda")
        ser = torch.zeros(nout // decim, device="cuda")

        def step(stream):
            r, n = P.pond_dedisperse_series(h, x, nsamp, subint, prof, nprof, decim, ser, ser.numel(), stream)
            assert r == nprof and n == ser.numel()
            assert P.pond_dedisperse_fold(h, None, 0, subint, prof[nprof:], 1, stream) == 1

        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            step(s)                      # eager reference (also grows every buffer)
        torch.cuda.synchronize()
        ref_p, ref_s = prof.clone(), ser.clone()

        g = torch.cuda.CUDAGraph()
        prof.zero_()
        ser.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            step(torch.cuda.current_stream())
        for rep in range(3):
            prof.fill_(-1.0)
            ser.fill_(-1.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(prof.cpu().numpy(), ref_p.cpu().numpy(), err_msg=f"replay {rep}")
            np.testing.assert_array_equal(ser.cpu().numpy(), ref_s.cpu().numpy(), err_msg=f"replay {rep}")
            # eager work between replays, on the same plan and stream
            with torch.cuda.stream(s):
                step(s)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(prof.cpu().numpy(), ref_p.cpu().numpy())
        del g
    finally:
        P.pond_plan_destroy(h)


def test_real_path_graph_replay_matches_eager():
    """The same for a real two-channel plan (fused middle pass)."""
    import torch
    import paper_1503_01405_amd as P

    nfft, dm, nbins, period, subint, decim = 1 << 19, 1.0, 128, synth.PERIOD_S, 1_000_000, 32
    nsamp = 3_000_002
    print(f"case: real graph replay nfft=2^19 nsamp={nsamp}", flush=True)
    x = torch.from_numpy(synth.white_stream_int8(22, nsamp)).to("cuda")
    h = P.pond_real_plan_create(F0, BW, dm, nfft, nbins, period, P.POND_MIXED_VALU, 0, "usb")
    try:
        nprof, nout = P.pond_real_expect(h, nsamp, subint)
        prof = torch.zeros((nprof + 1, nbins), device="cuda")
        ser = torch.zeros(nout // decim, device="cuda")

        def step(stream):
            r, n = P.pond_real_dedisperse(h, x, nsamp, subint, prof, nprof, decim, ser, ser.numel(), stream)
            assert r == nprof and n == ser.numel()
            assert P.pond_real_dedisperse(h, None, 0, subint, prof[nprof:], 1, decim, None, 0, stream)[0] == 1

        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            step(s)
        torch.cuda.synchronize()
        ref_p, ref_s = prof.clone(), ser.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step(torch.cuda.current_stream())
        for rep in range(3):
            prof.fill_(-1.0)
            ser.fill_(-1.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(prof.cpu().numpy(), ref_p.cpu().numpy(), err_msg=f"replay {rep}")
            np.testing.assert_array_equal(ser.cpu().numpy(), ref_s.cpu().numpy(), err_msg=f"replay {rep}")
            with torch.cuda.stream(s):
                step(s)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(prof.cpu().numpy(), ref_p.cpu().numpy())
        del g
    finally:
        P.pond_plan_destroy(h)
