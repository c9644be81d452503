"""Shared helpers of the GPU parity tests: run a stream through the C ABI
(via the ctypes binding) and through the FP64 oracle, and compare."""
from __future__ import annotations

import numpy as np

import oracle as O
import synth

F0, BW = 326.5, 16.0


def dispersed_pulsar_stream(seed, nsamp, dm, nfft_gen=1 << 20, period=synth.PERIOD_S):
    """Pulsed noise dispersed with the ISM response (oracle forward model),
    quantised to int8 -- the input recipe of the small workload."""
    fs = BW * 1e6
    pad_lo, pad_hi = O.disperse_pads(F0, BW, dm)
    z = synth.pulsed_noise(seed, pad_lo + nsamp + pad_hi, first_index=-pad_lo, fs_hz=fs,
                           period_s=period)
    while 2 * (pad_lo + pad_hi) >= nfft_gen:
        nfft_gen *= 2
    return synth.quantize_int8(O.disperse(z, F0, BW, dm, nfft_gen))


def gpu_run(iq, dm, nfft, nbins, period, subint=0, decim=16, precision="fp32",
            chunks=None, max_batch=0, want_series=True, taper=0.0):
    """Stream iq (numpy int8) through a plan in the given chunk sizes (one
    call if None), flush, and return (profiles [k, nbins], series) as numpy."""
    import torch
    from paper_1503_01405_amd import Plan
    dev = torch.device("cuda")
    x = torch.from_numpy(np.ascontiguousarray(iq)).to(dev)
    nsamp = iq.size // 2
    if chunks is None:
        chunks = [nsamp]
    plan = Plan(F0, BW, dm, nfft, nbins, period, precision=precision, max_batch=max_batch,
                subint_nsamp=subint, decim=decim, taper_alpha=taper)
    profs, sers = [], []
    pos = 0
    for c in chunks:
        c = min(c, nsamp - pos)
        if c < 0:
            break
        pr, se = plan.process(x[2 * pos:2 * (pos + c)], want_series=want_series)
        profs.append(pr.cpu().numpy())
        if se is not None:
            sers.append(se.cpu().numpy())
        pos += c
    assert pos == nsamp, (pos, nsamp)
    profs.append(plan.flush(device=dev).cpu().numpy())
    torch.cuda.synchronize()
    plan.close()
    prof = np.concatenate(profs, axis=0) if profs else np.zeros((0, nbins), np.float32)
    ser = np.concatenate(sers) if sers else np.zeros(0, np.float32)
    return prof, ser


def oracle_run(iq, dm, nfft, nbins, period, subint=0, decim=16, taper=0.0):
    """Oracle profiles in the order the library emits them (completed
    sub-integrations, then the open one at the end of the stream) and the
    full decimated series."""
    r = O.run(iq, F0, BW, dm, nfft, nbins, period, subint_nsamp=subint, decim=decim, workers=8,
              taper_alpha=taper)
    n_out = r["n_out"]
    if subint > 0:
        k = r["complete"]
        rows = [r["profiles"][i] for i in range(k)]
        if n_out > k * subint:
            rows.append(r["profiles"][k])
    else:
        rows = [r["profiles"][0]] if n_out > 0 else []
    prof = np.array(rows).reshape(-1, nbins)
    return prof, r["series"], r


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / d) if d > 0 else float(np.linalg.norm(a - b))


def profile_rel_l2(a, b):
    """Maximum over sub-integrations of the per-profile relative L2 error."""
    assert a.shape == b.shape, (a.shape, b.shape)
    return max((rel_l2(a[i], b[i]) for i in range(a.shape[0])), default=0.0)


EPS_HALF = 5e-3     # bound on the per-sample relative error of a float16-form detected power
BIAS_TOL = 2e-5     # systematic power gain allowed in any form


def power_gain(prof, oprof, cnts):
    """Total folded power of the GPU profiles over the oracle's: each bin's
    mean weighted by its count (the oracle's), summed over every profile.
    A systematic gain of the arithmetic shows here undiluted, while
    zero-mean rounding noise averages out over all outputs."""
    prof = np.asarray(prof, np.float64)
    oprof = np.asarray(oprof, np.float64)
    cnts = np.asarray(cnts, np.float64)[:prof.shape[0]]
    return float((prof * cnts).sum() / (oprof * cnts).sum())


def bias_tol(n_out):
    """Allowed |power gain - 1| over n_out outputs: BIAS_TOL plus three
    standard deviations of the float16 rounding noise of their mean."""
    return BIAS_TOL + 3 * EPS_HALF / np.sqrt(max(1, n_out))
