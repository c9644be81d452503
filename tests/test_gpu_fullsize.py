"""The 60 s DM-50 stream at its full size, in the launch configuration the
benchmark times (one call over all 960,000,000 samples, blocks of 2^23 in
launches of the default batch, 1024 bins per 10 s, 1 us series), against
the FP64 oracle run over the same whole stream:

* every profile (5 complete sub-integrations and the open one), element by
  element: relative L2 at most 1e-4 in the packed-float16 form (the stated
  accuracy target, flat: no noise allowance) and 1e-6 in float32;
* the systematic power gain (total folded power over the oracle's) within
  2e-5 plus the float16 noise of a mean over 9.5e8 outputs (5e-7);
* the whole 1 us series (59.5 million values): relative L2 1e-2 / 1e-5;
* each sub-integration's profile means times the oracle's counts sum to its
  series total (fold and series of the GPU agree with each other).
"""
import time

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import BW, F0, bias_tol, power_gain, rel_l2

pytestmark = pytest.mark.gpu

DM, NFFT, NBINS, PERIOD = 50.0, 1 << 23, 1024, synth.PERIOD_S
NSAMP, SUBINT, DECIM = 960_000_000, 160_000_000, 16
PROFILE_TOL = {"fp32": 1e-6, "half": 1e-4, "mixed": 1e-4}
SERIES_TOL = {"fp32": 1e-5, "half": 1e-2, "mixed": 1e-2}


@pytest.fixture(scope="module")
def stream():
    print("case: full 60 s stream, generating", flush=True)
    return synth.pulsed_stream_int8(2, NSAMP)


@pytest.fixture(scope="module")
def oracle_full(stream):
    print("case: full 60 s stream, oracle (about a minute on 16 cores)", flush=True)
    t0 = time.perf_counter()
    r = O.run(stream, F0, BW, DM, NFFT, NBINS, PERIOD, subint_nsamp=SUBINT, decim=DECIM, workers=16)
    print(f"oracle: {r['n_out']} outputs in {time.perf_counter() - t0:.1f} s", flush=True)
    return r


@pytest.mark.parametrize("precision", ["half", "mixed", "fp32"])
def test_full_stream_profiles_and_series_vs_oracle(stream, oracle_full, precision):
    import torch
    import paper_1503_01405_amd as P
    r = oracle_full
    n_out, cnt = r["n_out"], r["cnts"]
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
    want = r["profiles"]
    assert prof.shape == want.shape == cnt.shape == (6, NBINS)
    assert ser.size == r["series"].size == n_out // DECIM
    for s in range(prof.shape[0]):
        e = rel_l2(prof[s], want[s])
        print(f"subint {s}: profile rel-L2 {e:.3e}", flush=True)
        assert e <= PROFILE_TOL[precision], (s, e)
    gain = power_gain(prof, want, cnt)
    es = rel_l2(ser, r["series"])
    print(f"{precision}: power gain {gain - 1:+.3e}, series rel-L2 {es:.3e}", flush=True)
    assert abs(gain - 1) <= bias_tol(n_out)
    assert es <= SERIES_TOL[precision]
    # the fold and the series of the GPU agree: per sub-integration, the
    # sum of mean x count equals the sum of the series values
    per = SUBINT // DECIM
    for s in range(cnt.shape[0]):
        total_prof = float((prof[s] * cnt[s]).sum())
        total_ser = float(ser[s * per:min((s + 1) * per, ser.size)].sum())
        assert abs(total_prof - total_ser) / total_ser < 1e-5, s
    assert cnt.sum() == n_out
