"""Incoherent (AID) mode on the GPU against the oracle: channel delays,
dedispersed series and folded profile, element by element, for several
channel counts, integrations and DMs, including ragged stream lengths."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import BW, F0, dispersed_pulsar_stream, rel_l2

pytestmark = pytest.mark.gpu

# (nchan, nint, dm, nbins, period, nsamp)
CASES = [
    (64, 8, 5.0, 64, 0.02, 4_000_000),
    (256, 2, 0.0, 32, 3.3e-3, 1_000_003),
    (1024, 4, 50.0, 1024, 0.0891, 24_000_001),
    (4096, 1, 12.5, 128, 0.25, 9_000_000),
    (128, 16, 1.0, 100, 7.1e-3, 2_500_017),
]


def _gpu_aid(iq, nchan, nint, dm, nbins, period):
    import torch
    import paper_1503_01405_amd as P
    x = torch.from_numpy(iq).to("cuda")
    h = P.pond_aid_create(F0, BW, dm, nchan, nint, nbins, period)
    try:
        geo = P.pond_aid_geometry(h, iq.size // 2)
        prof = torch.zeros(nbins, device="cuda")
        ser = torch.zeros(max(geo["n_series"], 1), device="cuda")
        n = P.pond_aid_run(h, x, iq.size // 2, prof, ser, ser.numel())
        torch.cuda.synchronize()
        assert n == geo["n_series"], (n, geo)
        return prof.cpu().numpy(), ser[:n].cpu().numpy(), geo
    finally:
        P.pond_aid_destroy(h)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"c{c[0]}_i{c[1]}_dm{c[2]}")
def test_aid_parity(case):
    nchan, nint, dm, nbins, period, nsamp = case
    print(f"case: aid nchan={nchan} nint={nint} dm={dm} nbins={nbins} nsamp={nsamp}", flush=True)
    iq = dispersed_pulsar_stream(21, nsamp, dm, period=period) if dm > 0 else synth.white_stream_int8(21, nsamp)
    ref = O.aid_run(iq, F0, BW, dm, nchan, nint, nbins, period)
    prof, ser, geo = _gpu_aid(iq, nchan, nint, dm, nbins, period)
    assert geo["d_min"] == ref["d_min"] and geo["d_max"] == int(ref["delays"].max())
    assert geo["n_series"] == ref["series"].size and geo["n_spectra"] == ref["filterbank"].shape[0]
    es, ep = rel_l2(ser, ref["series"]), rel_l2(prof, ref["profile"])
    print(f"aid: series rel-L2 {es:.3e} profile rel-L2 {ep:.3e}")
    assert es <= 1e-5 and ep <= 1e-5


def test_aid_too_short_stream():
    """Fewer integrated samples than the delay span: no outputs, empty bins."""
    nchan, nint, dm = 1024, 4, 50.0
    iq = synth.white_stream_int8(3, 2_000_000)  # 488 integrated samples < 746 of delay span
    prof, ser, geo = _gpu_aid(iq, nchan, nint, dm, 64, 0.0891)
    assert geo["n_series"] == 0 and ser.size == 0 and np.all(prof == 0)
