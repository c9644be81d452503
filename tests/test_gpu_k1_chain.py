"""The chained column pass, through the C ABI.

Where blocks overlap by half (hop = N / 2: a discard of N / 2, the
production shape and every DM-search group), K1 gives each workgroup its
column tile in up to four consecutive blocks and loads only the second half
of every block after the first, the first half being the previous block's
second half, already in registers.  A launch in which a block straddles the
end of the carried tail uses the one-block-per-workgroup pass.  The values
and the arithmetic are the same (the matrix-core form takes the packed-
float16 column pass wherever blocks overlap by half, chained or not), so:
  * a stream at four blocks per launch (chained) equals the same stream at
    one block per launch (never chained) bit for bit, profiles and series;
  * the stream cut into calls whose ends fall inside blocks (launches that
    straddle the tail, and chains that start after a carried tail) equals
    the stream in one call bit for bit;
  * the profiles match the oracle (Sec. 3.7) at the form's tolerance.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import bias_tol, dispersed_pulsar_stream, gpu_run, oracle_run, power_gain, profile_rel_l2
from test_gpu_parity import TOL, profile_tol

pytestmark = pytest.mark.gpu

# (nfft, DM, samples): discard N / 2 at 326.5 MHz, 16 MHz
CASES = {"2^12": (1 << 12, 0.03, 200_000), "2^16": (1 << 16, 0.5, 1_500_000), "2^18": (1 << 18, 2.0, 3_000_000),
         "2^20": (1 << 20, 8.0, 12_000_000)}
FORMS = ["fp32", "mixed_valu", "half", "mixed", "bf16"]
NBINS, SUBINT = 256, 2_000_000


def bits(x):
    return np.ascontiguousarray(x).view(np.uint32)


@pytest.fixture(scope="module")
def streams():
    return {k: dispersed_pulsar_stream(21, ns, dm) for k, (n, dm, ns) in CASES.items()}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", FORMS)
def test_chained_equals_unchained(streams, case, precision):
    nfft, dm, ns = CASES[case]
    print(f"case: K1 chain {case} DM {dm} {precision}", flush=True)
    iq = streams[case]
    p4, s4 = gpu_run(iq, dm, nfft, NBINS, synth.PERIOD_S, subint=SUBINT, precision=precision, max_batch=4)
    p1, s1 = gpu_run(iq, dm, nfft, NBINS, synth.PERIOD_S, subint=SUBINT, precision=precision, max_batch=1)
    assert p4.shape == p1.shape and s4.shape == s1.shape
    assert np.array_equal(bits(p4), bits(p1))
    assert np.array_equal(bits(s4), bits(s1))
    # calls ending inside blocks: 0.37, 1.1 and 2.3 hops, then the rest
    hop = nfft // 2
    chunks = [int(0.37 * hop), int(1.1 * hop), int(2.3 * hop), ns]
    pc, sc = gpu_run(iq, dm, nfft, NBINS, synth.PERIOD_S, subint=SUBINT, precision=precision, max_batch=4,
                     chunks=chunks)
    assert np.array_equal(bits(pc), bits(p4))
    assert np.array_equal(bits(sc), bits(s4))


@pytest.mark.parametrize("precision", ["fp32", "half"])
def test_chained_oracle_parity(streams, precision):
    nfft, dm, ns = CASES["2^20"]
    print(f"case: K1 chain oracle 2^20 DM {dm} {precision}", flush=True)
    iq = streams["2^20"]
    prof, ser = gpu_run(iq, dm, nfft, NBINS, synth.PERIOD_S, subint=SUBINT, precision=precision, max_batch=4)
    oprof, oser, r = oracle_run(iq, dm, nfft, NBINS, synth.PERIOD_S, subint=SUBINT, decim=16)
    assert prof.shape == oprof.shape and ser.shape == oser.shape
    err = profile_rel_l2(prof, oprof)
    assert err < profile_tol(precision, r["n_out"], SUBINT, NBINS), err
    assert np.linalg.norm(ser - oser) / np.linalg.norm(oser) < TOL[precision][1]
    gain = power_gain(prof, oprof, r["cnts"])
    assert abs(gain - 1.0) < bias_tol(r["n_out"]), gain


@pytest.mark.parametrize("precision", ["fp32", "mixed_valu"])
def test_chained_real_input_equals_unchained(precision):
    """The real two-channel input (Sec. 3.7's AIP: 4 bytes per packed
    element) through the chained pass: real blocks of 2^20 (packed 2^19) at
    DM 3.1 overlap by half."""
    from test_real_path import gpu_real_run, real_stream
    print(f"case: K1 chain real input lsb 2^20 DM 3.1 {precision}", flush=True)
    raw = real_stream(41, 3_000_002, 3.1, 3.3e-2, "lsb")
    p4, s4 = gpu_real_run(raw, 3.1, 1 << 20, 256, 3.3e-2, "lsb", precision=precision, max_batch=4)
    p1, s1 = gpu_real_run(raw, 3.1, 1 << 20, 256, 3.3e-2, "lsb", precision=precision, max_batch=1)
    assert p4.shape == p1.shape and s4.shape == s1.shape
    assert np.array_equal(bits(p4), bits(p1))
    assert np.array_equal(bits(s4), bits(s1))
