"""Queued fold reductions, through the C ABI.

A K3 launch whose per-workgroup fold partials fit in a quarter of the
partial buffers writes them there and queues its reduction; four queued
reductions run as one launch.  A launch whose partials need the whole
buffers first runs the queued ones.  Here (blocks of 2^20, 256 workgroups at
four blocks per launch, 1,050 bins, 5 M-output sub-integrations) a launch
inside one sub-integration has 1,050 histogram entries per workgroup and is
queued, one that straddles a boundary has 2,100 and is reduced at once, so
the two kinds alternate along the stream.  The fold is an integer sum, so
every schedule gives the same bits: the stream at four blocks per launch
must equal the stream at one block per launch (every launch queued) bit for
bit, profiles and series, and match the oracle (Sec. 3.7) at the form's
tolerance.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import bias_tol, dispersed_pulsar_stream, gpu_run, oracle_run, power_gain, profile_rel_l2
from test_gpu_parity import TOL, profile_tol

pytestmark = pytest.mark.gpu

NFFT, NBINS, SUBINT, DM = 1 << 20, 1050, 5_000_000, 1.0


@pytest.fixture(scope="module")
def stream_iq():
    # 3.5 s at 16 Msps, pulsed noise dispersed at DM 1 (seed 11)
    return dispersed_pulsar_stream(11, 56_000_000, DM)


@pytest.fixture(scope="module")
def stream_oracle(stream_iq):
    return oracle_run(stream_iq, DM, NFFT, NBINS, synth.PERIOD_S, subint=SUBINT, decim=16)


@pytest.mark.parametrize("precision", ["fp32", "half"])
def test_queued_and_immediate_reductions_agree(stream_iq, stream_oracle, precision):
    print(f"case: fold queue N=2^20 {NBINS} bins subint {SUBINT} {precision}", flush=True)
    p4, s4 = gpu_run(stream_iq, DM, NFFT, NBINS, synth.PERIOD_S, subint=SUBINT, precision=precision, max_batch=4)
    p1, s1 = gpu_run(stream_iq, DM, NFFT, NBINS, synth.PERIOD_S, subint=SUBINT, precision=precision, max_batch=1)
    assert p4.shape == p1.shape and s4.shape == s1.shape
    assert np.array_equal(p4.view(np.uint32), p1.view(np.uint32))
    assert np.array_equal(s4.view(np.uint32), s1.view(np.uint32))
    oprof, oser, r = stream_oracle
    assert p4.shape == oprof.shape
    err = profile_rel_l2(p4, oprof)
    assert err < profile_tol(precision, r["n_out"], SUBINT, NBINS), err
    assert np.linalg.norm(s4 - oser) / np.linalg.norm(oser) < TOL[precision][1]
    gain = power_gain(p4, oprof, r["cnts"])
    assert abs(gain - 1.0) < bias_tol(r["n_out"]), gain
