"""The 60 s DM-50 stream at its full size, in the launch configuration the
benchmark times (one call over all 960,000,000 samples, blocks of 2^23 in
launches of the default batch, 1024 bins per 10 s, 1 us series): sampled
blocks of the series against the oracle block by block, and, over the whole
stream, each sub-integration's profile against its series (the sum of mean
x count over bins equals the sum of the series values of that
sub-integration, with the counts from the oracle's fold phase)."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import BW, F0, rel_l2

pytestmark = pytest.mark.gpu

DM, NFFT, NBINS, PERIOD = 50.0, 1 << 23, 1024, synth.PERIOD_S
NSAMP, SUBINT, DECIM = 960_000_000, 160_000_000, 16
SERIES_TOL = {"fp32": 1e-5, "half": 1e-2}


@pytest.fixture(scope="module")
def stream():
    print("case: full 60 s stream, generating", flush=True)
    return synth.pulsed_stream_int8(2, NSAMP)


@pytest.fixture(scope="module")
def counts():
    """Outputs per (sub-integration, bin) of the whole stream, from the
    oracle's fold phase, in chunks."""
    g = O.plan_geometry(F0, BW, DM, NFFT)
    n_out = O.n_blocks(NSAMP, NFFT, g["hop"]) * g["hop"]
    nsub = (n_out - 1) // SUBINT + 1
    c = np.zeros((nsub, NBINS), dtype=np.int64)
    step = 1 << 24
    for m0 in range(0, n_out, step):
        m = np.arange(m0, min(m0 + step, n_out), dtype=np.int64)
        b = O.fold_bins(m, g["n_front"], PERIOD, BW * 1e6, NBINS)
        c += np.bincount((m // SUBINT) * NBINS + b, minlength=nsub * NBINS).reshape(nsub, NBINS)
    return g, n_out, c


@pytest.mark.parametrize("precision", ["half", "fp32"])
def test_full_stream_sampled_blocks_and_profiles(stream, counts, precision):
    import torch
    import paper_1503_01405_amd as P
    g, n_out, cnt = counts
    hop = g["hop"]
    print(f"case: full stream {precision}", flush=True)
    x = torch.from_numpy(stream).to("cuda")
    plan = P.Plan(F0, BW, DM, NFFT, NBINS, PERIOD, precision=precision, subint_nsamp=SUBINT, decim=DECIM)
    prof, ser = plan.process(x)
    last = plan.flush(device=x.device)
    torch.cuda.synchronize()
    prof = np.concatenate([prof.cpu().numpy(), last.cpu().numpy()]).astype(np.float64)
    ser = ser.cpu().numpy().astype(np.float64)
    plan.close()
    del x
    assert prof.shape == cnt.shape and ser.size == n_out // DECIM
    # sampled blocks against the oracle, element by element
    for b in (0, 113, n_out // hop - 1):
        xs = O.unpack(stream[2 * b * hop:2 * (b * hop + NFFT)])
        y, _ = O.dedisperse(xs, F0, BW, DM, NFFT, first_block=0, nblocks=1, workers=16)
        want = O.decimate(O.detect(y), DECIM)
        got = ser[b * hop // DECIM:(b + 1) * hop // DECIM]
        e = rel_l2(got, want)
        print(f"block {b}: series rel-L2 {e:.3e}", flush=True)
        assert e <= SERIES_TOL[precision], (b, e)
    # every sub-integration: profile means x counts against its series
    per = SUBINT // DECIM
    for s in range(cnt.shape[0]):
        total_prof = float((prof[s] * cnt[s]).sum())
        total_ser = float(ser[s * per:min((s + 1) * per, ser.size)].sum())
        e = abs(total_prof - total_ser) / total_ser
        print(f"subint {s}: profile-vs-series {e:.2e}", flush=True)
        assert e < 1e-5, (s, e)
    assert cnt.sum() == n_out
