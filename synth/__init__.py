"""Seeded synthetic baseband streams shaped like the Ooty Radio Telescope's
pulsar data (single polarisation, 8-bit samples, 16 MHz complex baseband at
326.5 MHz; Sec. 2, Sec. 3.1 and Sec. 4 of Naidu et al., arXiv:1503.01405).

This module holds only the input recipe: Gaussian noise, a periodic pulse
envelope and the 8-bit quantiser.  It contains none of the dedispersion
arithmetic (no FFT, no chirp, no detection, no fold), so both the FP64 oracle
and the GPU path can take their inputs from it without sharing any of the
method's code.  Interstellar dispersion of a test stream is the oracle's
forward model and lives there.

Recipe (one stream):
  * each complex sample is I + iQ with I, Q independent N(0, sigma^2),
    sigma = 20.  Samples are drawn in chunks of 2^22: chunk c (samples
    [c 2^22, (c+1) 2^22)) comes from ``standard_normal((n, 2))`` of a numpy
    Generator on ``PCG64(seed).jumped(c)``, so chunks can be drawn in
    parallel and any sample range is reproducible on its own;
  * a pulse of Gaussian shape (full width at half maximum ``fwhm_s``) centred
    at rotational phase ``phase0`` multiplies the noise amplitude by
    sqrt(1 + peak * g(t)), so the expected power is (1 + peak * g) times the
    noise power;
  * quantisation rounds half to even and clips to the int8 range
    [-128, 127]; I and Q are interleaved, I first.

Real two-channel recipe (the receiver's own sampling, Sec. 3.1): a real
voltage sampled at twice the bandwidth (the I component of the stream
above, at that rate) is given to two channels A and B as x/2 plus
independent N(0, noise^2) receiver noise each, quantised as above and
interleaved A0 B0 A1 B1 ...
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

SIGMA = 20.0          # per-component noise standard deviation (8-bit counts)
F0_MHZ = 326.5        # ORT centre frequency
BW_MHZ = 16.0         # complex bandwidth == complex sample rate in Msps
PERIOD_S = 0.0891     # synthetic pulsar period
FWHM_S = 1.0e-3       # pulse full width at half maximum
PEAK = 3.0            # pulse peak power in units of the noise power
PHASE0 = 0.5          # rotational phase of the pulse centre

_CHUNK_LOG2 = 22
_CHUNK = 1 << _CHUNK_LOG2
_THREADS = max(1, min(16, os.cpu_count() or 1))


def pulse_gain(sample_index, fs_hz, period_s=PERIOD_S, fwhm_s=FWHM_S,
               peak=PEAK, phase0=PHASE0):
    """Amplitude multiplier sqrt(1 + peak*g(t)) at t = sample_index / fs_hz.

    g is a unit-height Gaussian in time of full width at half maximum
    ``fwhm_s`` centred on rotational phase ``phase0`` of every period.
    """
    t = np.asarray(sample_index, dtype=np.float64) / fs_hz
    ph = t / period_s - phase0
    dt = (ph - np.rint(ph)) * period_s          # signed offset from the nearest pulse centre
    g = np.exp(-4.0 * math.log(2.0) * (dt / fwhm_s) ** 2)
    return np.sqrt(1.0 + peak * g)


def pulse_power_shape(sample_index, fs_hz, period_s=PERIOD_S, fwhm_s=FWHM_S,
                      peak=PEAK, phase0=PHASE0):
    """Expected power envelope 1 + peak*g(t) (the square of ``pulse_gain``)."""
    return pulse_gain(sample_index, fs_hz, period_s, fwhm_s, peak, phase0) ** 2


def _chunk_normals(seed: int, c: int, n: int):
    """The first n (I, Q) standard-normal pairs of chunk c."""
    g = np.random.Generator(np.random.PCG64(seed).jumped(c))
    return g.standard_normal((n, 2))


def _for_chunks(nsamp: int, fn):
    """Call fn(c, start, stop) for every chunk overlapping [0, nsamp), on a
    thread pool (numpy's generators and ufuncs release the GIL)."""
    nch = (nsamp + _CHUNK - 1) >> _CHUNK_LOG2
    spans = [(c, c << _CHUNK_LOG2, min(nsamp, (c + 1) << _CHUNK_LOG2)) for c in range(nch)]
    if len(spans) <= 1 or _THREADS == 1:
        for sp in spans:
            fn(*sp)
        return
    with ThreadPoolExecutor(_THREADS) as ex:
        list(ex.map(lambda sp: fn(*sp), spans))


def noise(seed: int, nsamp: int, sigma: float = SIGMA):
    """Complex128 Gaussian noise I + iQ, each component N(0, sigma^2)."""
    out = np.empty(nsamp, dtype=np.complex128)

    def fill(c, s, e):
        d = _chunk_normals(seed, c, e - s)
        out[s:e].real = d[:, 0] * sigma
        out[s:e].imag = d[:, 1] * sigma

    _for_chunks(nsamp, fill)
    return out


def pulsed_noise(seed: int, nsamp: int, first_index: int = 0,
                 fs_hz: float = BW_MHZ * 1e6, period_s: float = PERIOD_S,
                 fwhm_s: float = FWHM_S, peak: float = PEAK,
                 phase0: float = PHASE0, sigma: float = SIGMA):
    """Undispersed complex128 stream: noise times the pulse gain.

    Sample i of the result sits at time (first_index + i) / fs_hz, so a
    stream padded in front for a later dispersion step keeps its pulse phase
    referenced to the first sample the user keeps.
    """
    z = noise(seed, nsamp, sigma)
    idx = np.arange(first_index, first_index + nsamp, dtype=np.int64)
    z *= pulse_gain(idx, fs_hz, period_s, fwhm_s, peak, phase0)
    return z


def quantize_int8(z):
    """Interleaved int8 I/Q: round half to even, clip to [-128, 127]."""
    z = np.asarray(z)
    out = np.empty(2 * z.size, dtype=np.int8)
    out[0::2] = np.clip(np.rint(z.real), -128, 127).astype(np.int8)
    out[1::2] = np.clip(np.rint(z.imag), -128, 127).astype(np.int8)
    return out


def pulsed_stream_int8(seed: int, nsamp: int, fs_hz: float = BW_MHZ * 1e6,
                       period_s: float = PERIOD_S, fwhm_s: float = FWHM_S,
                       peak: float = PEAK, phase0: float = PHASE0,
                       sigma: float = SIGMA):
    """Undispersed pulsed noise quantised to int8, built chunk by chunk.

    Equal to ``quantize_int8(pulsed_noise(seed, nsamp, ...))`` but never
    holds more than a few chunks in float64, so a 60 s stream (1.92 GB of
    int8) can be built on a host with modest memory.
    """
    out = np.empty(2 * nsamp, dtype=np.int8)

    def fill(c, s, e):
        d = _chunk_normals(seed, c, e - s)
        gain = pulse_gain(np.arange(s, e, dtype=np.int64), fs_hz, period_s,
                          fwhm_s, peak, phase0)
        d *= (sigma * gain)[:, None]
        np.rint(d, out=d)
        np.clip(d, -128, 127, out=d)
        out[2 * s:2 * e] = d.astype(np.int8).reshape(-1)

    _for_chunks(nsamp, fill)
    return out


def white_stream_int8(seed: int, nsamp: int, sigma: float = SIGMA):
    """Pure noise quantised to int8 (no pulse)."""
    out = np.empty(2 * nsamp, dtype=np.int8)

    def fill(c, s, e):
        d = _chunk_normals(seed, c, e - s) * sigma
        np.rint(d, out=d)
        np.clip(d, -128, 127, out=d)
        out[2 * s:2 * e] = d.astype(np.int8).reshape(-1)

    _for_chunks(nsamp, fill)
    return out


def pulsed_real_noise(seed: int, nsamp: int, first_index: int = 0,
                      fs_hz: float = 2 * BW_MHZ * 1e6, period_s: float = PERIOD_S,
                      fwhm_s: float = FWHM_S, peak: float = PEAK,
                      phase0: float = PHASE0, sigma: float = SIGMA):
    """Undispersed real float64 stream at the real sample rate: the I
    component of pulsed_noise."""
    return pulsed_noise(seed, nsamp, first_index, fs_hz, period_s, fwhm_s, peak, phase0, sigma).real.copy()


def two_channel_int8(x, seed: int, noise: float = 5.0):
    """Interleaved int8 A0 B0 A1 B1 ...: A, B = x/2 plus independent
    N(0, noise^2) noise each, rounded half to even and clipped."""
    x = np.asarray(x, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(2 * x.size, dtype=np.int8)
    for k in range(2):
        d = x / 2 + noise * rng.standard_normal(x.size)
        np.rint(d, out=d)
        np.clip(d, -128, 127, out=d)
        out[k::2] = d.astype(np.int8)
    return out
