"""Blocks of 2^25 and 2^27 samples (rows of 2^15 and 2^17, longer than one
workgroup transforms in LDS: the split middle pass) against the FP64
oracle, element by element, at DM 130 (smear about 7.9 million samples at
16 Msps: the block must be long for the hop to stay large).

Tolerances as in the other parity tests (relative L2): float32 profiles
1e-6, series 1e-5; float16 storage / arithmetic profiles 1e-4 (plus the
float16 noise allowance for the float16-arithmetic forms), series 1e-2;
power gain within bias_tol.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import EPS_HALF, bias_tol, gpu_run, oracle_run, power_gain, profile_rel_l2, rel_l2

pytestmark = pytest.mark.gpu

DM = 130.0
TOL = {"fp32": (1e-6, 1e-5), "mixed": (1e-4, 1e-2), "mixed_valu": (1e-4, 1e-2), "half": (1e-4, 1e-2)}


def _tol(precision, n_out, nbins):
    tp = TOL[precision][0]
    if precision in ("half", "mixed"):
        tp += 3 * EPS_HALF / np.sqrt(max(1.0, n_out / nbins))
    return tp, TOL[precision][1]


def _hop(nfft):
    import paper_1503_01405_amd as P
    return P.pond_geometry(326.5, 16.0, DM, nfft)[2]


@pytest.fixture(scope="module")
def case25():
    nfft = 1 << 25
    nsamp = nfft + 2 * _hop(nfft) + 12345  # three blocks and a ragged tail
    print(f"case: split nfft=2^25 dm={DM} nsamp={nsamp}, oracle", flush=True)
    iq = synth.white_stream_int8(25, nsamp)
    return iq, nfft, oracle_run(iq, DM, nfft, 1024, synth.PERIOD_S, subint=0, decim=16)


@pytest.mark.parametrize("precision", ["fp32", "half", "mixed", "mixed_valu"])
def test_split_2e25_parity(case25, precision):
    iq, nfft, (oprof, oser, r) = case25
    print(f"case: split nfft=2^25 {precision}", flush=True)
    prof, ser = gpu_run(iq, DM, nfft, 1024, synth.PERIOD_S, precision=precision)
    assert prof.shape == oprof.shape and ser.shape == oser.shape
    ep, es = profile_rel_l2(prof, oprof), rel_l2(ser, oser)
    gain = power_gain(prof, oprof, r["cnts"])
    tp, ts = _tol(precision, r["n_out"], 1024)
    print(f"{precision}: profile rel-L2 {ep:.3e} (tol {tp:.1e}) series rel-L2 {es:.3e} gain {gain - 1:+.2e}", flush=True)
    assert ep <= tp and es <= ts
    assert abs(gain - 1) <= bias_tol(r["n_out"])


def test_split_2e25_chunking_is_bitwise(case25):
    """The stream cut into uneven calls gives the same bits as one call
    (the carried tail feeds the split pass like any other block)."""
    iq, nfft, _ = case25
    nsamp = iq.size // 2
    print("case: split nfft=2^25 chunked fp32", flush=True)
    one = gpu_run(iq, DM, nfft, 1024, synth.PERIOD_S, precision="fp32")
    cut = gpu_run(iq, DM, nfft, 1024, synth.PERIOD_S, precision="fp32",
                  chunks=[nfft // 3, nfft, 7 * nfft // 5, nsamp])
    assert np.array_equal(one[0], cut[0]) and np.array_equal(one[1], cut[1])


@pytest.mark.parametrize("precision", ["fp32", "half"])
def test_split_2e27_parity(precision):
    """The longest block (2^27 = 2^17 x 2^10, sub-rows of 2^13 in 16
    columns): two blocks and a ragged tail."""
    nfft = 1 << 27
    nsamp = nfft + _hop(nfft) + 777
    print(f"case: split nfft=2^27 dm={DM} nsamp={nsamp} {precision}, oracle", flush=True)
    iq = synth.white_stream_int8(27, nsamp)
    oprof, oser, r = _oracle27(iq, nfft)
    prof, ser = gpu_run(iq, DM, nfft, 1024, synth.PERIOD_S, precision=precision)
    assert prof.shape == oprof.shape and ser.shape == oser.shape
    ep, es = profile_rel_l2(prof, oprof), rel_l2(ser, oser)
    gain = power_gain(prof, oprof, r["cnts"])
    tp, ts = _tol(precision, r["n_out"], 1024)
    print(f"{precision}: profile rel-L2 {ep:.3e} (tol {tp:.1e}) series rel-L2 {es:.3e} gain {gain - 1:+.2e}", flush=True)
    assert ep <= tp and es <= ts
    assert abs(gain - 1) <= bias_tol(r["n_out"])


_ORACLE27 = {}


def _oracle27(iq, nfft):
    key = (iq.size, nfft)
    if key not in _ORACLE27:
        _ORACLE27.clear()
        _ORACLE27[key] = oracle_run(iq, DM, nfft, 1024, synth.PERIOD_S, subint=0, decim=16)
    return _ORACLE27[key]
