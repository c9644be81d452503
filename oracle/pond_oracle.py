"""FP64 CPU oracle for overlap-save coherent dedispersion, detection,
decimation and folding of complex baseband voltages -- the pulsar mode
("PCD") of PONDER, Naidu, Joshi, Manoharan & Krishnakumar,
"PONDER - A real time software backend for pulsar and IPS observations at
the Ooty Radio Telescope", arXiv:1503.01405.

THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the
package smoke check and the CPU-baseline leg of the benchmark may import it.
The GPU library neither imports nor links anything from here, and nothing
here imports the GPU library.

Everything is plain numpy/scipy in float64/complex128, written step by step
in the order the paper describes the method (Sec. 3.7 and Fig. 6: spectrum,
multiply by the inverse ISM response of Eq. (4), inverse transform, series,
fold).  The paper leaves several points open; the readings taken here are:

  C1  dispersion constant: 1/2.41e-4 s MHz^2 per unit DM (the constant of
      Eq. (1)); the chirp phase is DM f^2 / (2.41e-10 f0^2 (f0+f)) turns
      with f, f0 in MHz.  Eq. (4) as printed (8.3e3 pi) is short of the
      1e6 that turns MHz into Hz.
  C2  sign: numpy's forward transform is exp(-2 pi i k n / N); upper-side
      baseband (baseband f is sky f0 + f).  The ISM response is
      exp(+2 pi i turns) and dedispersion multiplies by its inverse
      exp(-2 pi i turns).
  C3  outputs are referred to arrival at f0.  Per block the first
      n_front = ceil(delta_hi fs) samples and the last discard - n_front
      samples are dropped, with s = ceil(delta_hi fs) + ceil(delta_lo fs)
      and discard = next_pow2(max(s, 16)) if that is <= N/2, otherwise s
      rounded up to a multiple of 16 (discard = 0 when s = 0).
  C4  taper: unit by default (the paper does not say which taper it
      uses).  Optional reading: a Tukey window over baseband frequency,
      w(f) = 1 for |f| <= (1 - alpha) bw/2 and
      w(f) = (1 + cos(pi (|f| - (1 - alpha) bw/2) / (alpha bw/2))) / 2
      beyond, falling to 0 at the band edge; it multiplies H^-1.
  C5  bin k = N/2 is the frequency -bw/2 (numpy fftfreq).
  C6  forward transform unnormalised, inverse with 1/N.
  C7  detection is |y|^2 with no baseline or bandpass correction.
  C8  the time series is the SUM of `decim` consecutive powers.
  C9  fold phase: output m is input sample m + n_front; with
      inv_pfs = 1 / (period_s * fs_hz),  x = (m + n_front) * inv_pfs,
      bin = min(floor((x - floor(x)) * nbins), nbins - 1), all in float64.
  C10 profile value = mean power per bin (sum / count, 0 for an empty bin).
  C11 sub-integration s holds outputs m in [s*S, (s+1)*S).
  C12 Eq. (1) read as N_min = 2 * smear / ts.
  C16 only fully covered blocks produce outputs.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

# C1: the dispersion constant of Eq. (1), in s MHz^2 cm^3 / pc.
DM_CONST_S = 1.0 / 2.41e-4
# The same constant with f in MHz and the result in turns (1e6 cycles per s*MHz).
DM_CONST_TURNS = 1.0 / 2.41e-10


# --------------------------------------------------------------------------
# Dispersion delays and the paper's design equations
# --------------------------------------------------------------------------
def dispersion_delay_s(f_mhz, f_ref_mhz, dm):
    """Cold-plasma delay of frequency f relative to f_ref, in seconds.

    Same form as Eq. (3) of Sec. 3.4 (4.15e6 (f_ref^-2 - f^-2) DM ms) with
    the sign chosen so that lower frequencies arrive later (positive delay).
    """
    f = np.asarray(f_mhz, dtype=np.float64)
    return DM_CONST_S * dm * (1.0 / (f * f) - 1.0 / (f_ref_mhz * f_ref_mhz))


def residual_smear_ms(df_ch_mhz, f_ch_mhz, dm):
    """Eq. (2), Sec. 3.4: dispersion smear inside one channel, in ms."""
    return 8.3e6 * df_ch_mhz * dm / f_ch_mhz ** 3


def fft_length_eq1(f_hi_mhz, df_mhz, dm, ts_s):
    """Eq. (1), Sec. 3.2, read as N = 2 * smear / ts (reading C12).

    The printed equation puts the 2 on each frequency term; the reading
    multiplies the full band smear (f_h - df)^-2 - f_h^-2 by 2 DM /
    (2.41e-4 ts).
    """
    smear = (1.0 / (f_hi_mhz - df_mhz) ** 2 - 1.0 / f_hi_mhz ** 2) * dm / 2.41e-4
    return 2.0 * smear / ts_s


# --------------------------------------------------------------------------
# Plan geometry (reading C3)
# --------------------------------------------------------------------------
def plan_geometry(f0_mhz, bw_mhz, dm, nfft):
    """Sample rate, smear and overlap-save discard/hop for one plan.

    Sec. 3.7: the filter must be longer than the dispersion smear and the
    cyclic edges of the FFT convolution must be dropped.  Returns a dict;
    raises ValueError where no output would be produced.
    """
    if nfft <= 0 or nfft & (nfft - 1):
        raise ValueError("nfft must be a power of two")
    if not (bw_mhz > 0 and f0_mhz - bw_mhz / 2 > 0 and dm >= 0):
        raise ValueError("need bw > 0, f0 - bw/2 > 0 and dm >= 0")
    fs = bw_mhz * 1e6
    f_lo = f0_mhz - bw_mhz / 2
    f_hi = f0_mhz + bw_mhz / 2
    delta_lo = DM_CONST_S * dm * (1.0 / (f_lo * f_lo) - 1.0 / (f0_mhz * f0_mhz))
    delta_hi = DM_CONST_S * dm * (1.0 / (f0_mhz * f0_mhz) - 1.0 / (f_hi * f_hi))
    n_front = int(math.ceil(delta_hi * fs))
    n_back_min = int(math.ceil(delta_lo * fs))
    s = n_front + n_back_min
    if s == 0:
        discard = 0
    else:
        p2 = 1 << max(4, (s - 1).bit_length())
        discard = p2 if p2 <= nfft // 2 else ((s + 15) // 16) * 16
    hop = nfft - discard
    if hop <= 0:
        raise ValueError("nfft too short for the dispersion smear")
    return dict(fs=fs, delta_lo=delta_lo, delta_hi=delta_hi,
                smear_samples=s, n_front=n_front, discard=discard, hop=hop,
                nfft=nfft)


def n_blocks(nsamp, nfft, hop):
    """Number of overlap-save blocks fully covered by nsamp samples (C16)."""
    if nsamp < nfft:
        return 0
    return (nsamp - nfft) // hop + 1


# --------------------------------------------------------------------------
# The chirp of Eq. (4)
# --------------------------------------------------------------------------
def baseband_freqs_mhz(nfft, bw_mhz):
    """Baseband frequency of each FFT bin in MHz (reading C5)."""
    return sfft.fftfreq(nfft, d=1.0 / bw_mhz)


def chirp_turns(f_mhz, f0_mhz, dm):
    """Phase of the ISM response H(f0 + f) of Eq. (4), in turns (reading C1)."""
    f = np.asarray(f_mhz, dtype=np.float64)
    return dm * f * f / (2.41e-10 * f0_mhz * f0_mhz * (f0_mhz + f))


def ism_response(nfft, f0_mhz, bw_mhz, dm):
    """H sampled on the FFT grid: exp(+2 pi i turns) (reading C2)."""
    return np.exp(2j * np.pi * chirp_turns(baseband_freqs_mhz(nfft, bw_mhz), f0_mhz, dm))


def taper(f_mhz, bw_mhz, alpha):
    """The frequency-domain taper of the filter (reading C4): a Tukey window
    of edge fraction alpha over [-bw/2, bw/2]; alpha = 0 is the unit taper."""
    f = np.abs(np.asarray(f_mhz, dtype=np.float64))
    if alpha <= 0:
        return np.ones_like(f)
    flat = (1.0 - alpha) * bw_mhz / 2
    edge = alpha * bw_mhz / 2
    w = np.ones_like(f)
    m = f > flat
    w[m] = 0.5 * (1.0 + np.cos(np.pi * np.minimum(f[m] - flat, edge) / edge))
    return w


def dedispersion_chirp(nfft, f0_mhz, bw_mhz, dm, taper_alpha=0.0):
    """H^-1 on the FFT grid, exp(-2 pi i turns), times the taper: the
    multiplier of Sec. 3.7."""
    f = baseband_freqs_mhz(nfft, bw_mhz)
    return np.exp(-2j * np.pi * chirp_turns(f, f0_mhz, dm)) * taper(f, bw_mhz, taper_alpha)


# --------------------------------------------------------------------------
# The method, step by step
# --------------------------------------------------------------------------
def unpack(iq):
    """Interleaved int8 I/Q -> complex128 x = I + iQ, no offset, no scale."""
    iq = np.asarray(iq)
    x = np.empty(iq.size // 2, dtype=np.complex128)
    x.real = iq[0::2]
    x.imag = iq[1::2]
    return x


def dedisperse_block(x_block, chirp, n_front, hop, workers=None):
    """One overlap-save block: fft, multiply by H^-1 (unit taper, C4),
    inverse fft with 1/N (C6), keep y[n_front : n_front + hop] (C3)."""
    X = sfft.fft(x_block, workers=workers)
    y = sfft.ifft(X * chirp, workers=workers)
    return y[n_front:n_front + hop]


def dedisperse(x, f0_mhz, bw_mhz, dm, nfft, first_block=0, nblocks=None,
               batch=8, workers=None, hop=None, taper_alpha=0.0):
    """Dedispersed voltages of blocks [first_block, first_block + nblocks).

    Block b covers input samples [b*hop, b*hop + nfft); its kept outputs are
    outputs m = b*hop + j for j in [0, hop) (input sample m + n_front).
    `hop` may be given to impose a common block grid (it must not exceed the
    plan's own hop, so the kept window stays clear of the cyclic edges).
    Returns (y, m0) with y complex128 and m0 the output index of y[0].
    """
    g = plan_geometry(f0_mhz, bw_mhz, dm, nfft)
    n_front = g["n_front"]
    if hop is None:
        hop = g["hop"]
    elif not (0 < hop <= g["hop"]):
        raise ValueError("imposed hop must be in (0, plan hop]")
    total = n_blocks(x.size, nfft, hop)
    if nblocks is None:
        nblocks = total - first_block
    if first_block < 0 or first_block + nblocks > total:
        raise ValueError("block range not covered by the input")
    chirp = dedispersion_chirp(nfft, f0_mhz, bw_mhz, dm, taper_alpha)
    y = np.empty(nblocks * hop, dtype=np.complex128)
    for b0 in range(0, nblocks, batch):
        nb = min(batch, nblocks - b0)
        X = np.stack([x[(first_block + b0 + i) * hop:(first_block + b0 + i) * hop + nfft]
                      for i in range(nb)])
        X = sfft.fft(X, axis=1, workers=workers)
        X *= chirp
        Y = sfft.ifft(X, axis=1, workers=workers)
        y[b0 * hop:(b0 + nb) * hop] = Y[:, n_front:n_front + hop].reshape(-1)
    return y, first_block * hop


def detect(y):
    """Square-law detection p = |y|^2 (reading C7)."""
    return y.real * y.real + y.imag * y.imag


def decimate(p, decim):
    """Time series: sum of `decim` consecutive powers (reading C8, Sec. 4's
    integration from the 62.5 ns base resolution to 1 us)."""
    n = p.size // decim
    return p[:n * decim].reshape(n, decim).sum(axis=1)


def fold_bins(m, n_front, period_s, fs_hz, nbins):
    """Profile bin of output m (reading C9), float64 throughout."""
    inv_pfs = 1.0 / (period_s * fs_hz)
    x = (np.asarray(m, dtype=np.int64) + n_front).astype(np.float64) * inv_pfs
    frac = x - np.floor(x)
    b = np.floor(frac * nbins).astype(np.int64)
    return np.minimum(b, nbins - 1)


def fold(p, m0, n_front, period_s, fs_hz, nbins, subint_nsamp):
    """Sums and counts per (sub-integration, bin) of powers p of outputs
    m0, m0+1, ...  (Sec. 3.4.1 and Sec. 3.7: the fold thread folds the
    dedispersed series at the pulsar period and writes profiles
    periodically; readings C9-C11).  Returns (sums, counts, first_subint).
    """
    m = m0 + np.arange(p.size, dtype=np.int64)
    b = fold_bins(m, n_front, period_s, fs_hz, nbins)
    if subint_nsamp > 0:
        s = m // subint_nsamp
    else:
        s = np.zeros_like(m)
    if p.size == 0:
        return np.zeros((0, nbins)), np.zeros((0, nbins), dtype=np.int64), 0
    s0 = int(s[0])
    ns = int(s[-1]) - s0 + 1
    idx = (s - s0) * nbins + b
    sums = np.bincount(idx, weights=p, minlength=ns * nbins).reshape(ns, nbins)
    cnts = np.bincount(idx, minlength=ns * nbins).reshape(ns, nbins).astype(np.int64)
    return sums, cnts, s0


def profiles_from(sums, cnts):
    """Mean power per bin, 0 where a bin is empty (reading C10)."""
    out = np.zeros_like(sums)
    nz = cnts > 0
    out[nz] = sums[nz] / cnts[nz]
    return out


def run(iq, f0_mhz, bw_mhz, dm, nfft, nbins, period_s, subint_nsamp=0,
        decim=16, batch=8, workers=None, keep_power=False, hop=None, taper_alpha=0.0):
    """The whole path over one stream, every fully covered block.

    Returns a dict with
      geometry   the plan geometry
      n_out      number of outputs (fully covered blocks x hop)
      series     sum of `decim` consecutive powers, float64
      sums, cnts per (sub-integration, bin), all sub-integrations touched
      profiles   sums / cnts
      complete   number of leading sub-integrations that are complete
      power      the detected series at full resolution (if keep_power)
    """
    g = plan_geometry(f0_mhz, bw_mhz, dm, nfft)
    x = unpack(iq)
    n_front = g["n_front"]
    if hop is None:
        hop = g["hop"]
    nb = n_blocks(x.size, nfft, hop)
    n_out = nb * hop
    series = np.empty(n_out // decim, dtype=np.float64)
    ns_total = (max(n_out - 1, 0) // subint_nsamp + 1) if (subint_nsamp > 0 and n_out) else (1 if n_out else 0)
    sums = np.zeros((ns_total, nbins))
    cnts = np.zeros((ns_total, nbins), dtype=np.int64)
    power = np.empty(n_out) if keep_power else None
    for b0 in range(0, nb, batch):
        k = min(batch, nb - b0)
        y, m0 = dedisperse(x, f0_mhz, bw_mhz, dm, nfft, first_block=b0,
                           nblocks=k, batch=batch, workers=workers, hop=hop,
                           taper_alpha=taper_alpha)
        p = detect(y)
        series[m0 // decim:(m0 + p.size) // decim] = decimate(p, decim)
        s, c, s0 = fold(p, m0, n_front, period_s, g["fs"], nbins, subint_nsamp)
        sums[s0:s0 + s.shape[0]] += s
        cnts[s0:s0 + c.shape[0]] += c
        if keep_power:
            power[m0:m0 + p.size] = p
    complete = (n_out // subint_nsamp) if subint_nsamp > 0 else 0
    g = dict(g, hop=hop)
    return dict(geometry=g, n_out=n_out, series=series, sums=sums, cnts=cnts,
                profiles=profiles_from(sums, cnts), complete=complete,
                power=power)


# --------------------------------------------------------------------------
# Forward model used to build test streams (the inverse of the method)
# --------------------------------------------------------------------------
def disperse_pads(f0_mhz, bw_mhz, dm):
    """Samples the dispersing filter needs before and after each output:
    ceil(delta_lo fs) in front (low frequencies arrive later), ceil(delta_hi
    fs) behind."""
    g = plan_geometry(f0_mhz, bw_mhz, dm, 1 << 30)
    return int(math.ceil(g["delta_lo"] * g["fs"])), int(math.ceil(g["delta_hi"] * g["fs"]))


def disperse(z, f0_mhz, bw_mhz, dm, nfft):
    """Apply the ISM response H (reading C2) to an undispersed stream by
    overlap-save.  z covers pad_lo samples before and pad_hi samples after
    the part kept; the result has z.size - pad_lo - pad_hi samples."""
    pad_lo, pad_hi = disperse_pads(f0_mhz, bw_mhz, dm)
    hop = nfft - pad_lo - pad_hi
    if hop <= 0:
        raise ValueError("nfft too short to disperse")
    n_keep = z.size - pad_lo - pad_hi
    H = ism_response(nfft, f0_mhz, bw_mhz, dm)
    nb = -(-n_keep // hop)
    zp = np.zeros(nb * hop + pad_lo + pad_hi + nfft, dtype=np.complex128)
    zp[:z.size] = z
    out = np.empty(nb * hop, dtype=np.complex128)
    for b in range(nb):
        y = sfft.ifft(sfft.fft(zp[b * hop:b * hop + nfft]) * H)
        out[b * hop:(b + 1) * hop] = y[pad_lo:pad_lo + hop]
    return out[:n_keep]


# --------------------------------------------------------------------------
# DM-trial search (one stream folded at many trial DMs)
# --------------------------------------------------------------------------
def search_geometry(f0_mhz, bw_mhz, dms, nfft_min=1 << 20, nfft_max=1 << 23):
    """Per-trial FFT length and common block grid of a DM search.

    Reading: each trial takes discard_t by the plan rule (C3) and
    N_t = clamp(2 discard_t, nfft_min, nfft_max); trials with equal N_t form
    a group that shares one block grid with hop = N_t / 2 (every trial's
    kept window [n_front_t, n_front_t + hop) stays clear of the cyclic
    edges because discard_t <= N_t / 2), so the forward transform of a
    block is shared by the whole group.  Returns a list of dicts.
    """
    out = []
    for dm in dms:
        g = plan_geometry(f0_mhz, bw_mhz, dm, nfft_max)
        if g["discard"] > nfft_max // 2:
            raise ValueError(f"DM {dm}: smear too long for nfft_max")
        n = max(nfft_min, min(nfft_max, 2 * g["discard"]))
        gn = plan_geometry(f0_mhz, bw_mhz, dm, n)
        out.append(dict(dm=float(dm), nfft=n, n_front=gn["n_front"], hop=n // 2))
    return out


def search(iq, f0_mhz, bw_mhz, dms, nbins, period_s, nfft_min=1 << 20,
           nfft_max=1 << 23, workers=None):
    """Folded profile (mean power per bin over every output of the stream)
    of each trial DM, each trial dedispersed as in `run` with its own chirp
    and n_front on its group's block grid."""
    geo = search_geometry(f0_mhz, bw_mhz, dms, nfft_min, nfft_max)
    profs = []
    for t in geo:
        r = run(iq, f0_mhz, bw_mhz, t["dm"], t["nfft"], nbins, period_s,
                subint_nsamp=0, decim=16, workers=workers, hop=t["hop"])
        profs.append(r["profiles"][0] if r["n_out"] else np.zeros(nbins))
    return np.array(profs), geo


def profile_snr(profile, on_frac=0.1):
    """Peak signal-to-noise of a folded profile: (max - median) over the
    standard deviation of the bins outside the +-on_frac window around the
    peak."""
    p = np.asarray(profile, dtype=np.float64)
    n = p.size
    k = int(np.argmax(p))
    w = max(1, int(on_frac * n))
    mask = np.ones(n, dtype=bool)
    for d in range(-w, w + 1):
        mask[(k + d) % n] = False
    off = p[mask]
    return float((p[k] - np.median(off)) / off.std())


# --------------------------------------------------------------------------
# Incoherent dedispersion with an FFT filterbank (AID mode, Sec. 3.4 and
# Sec. 3.4.1): spectra of consecutive blocks, squared and added to the
# wanted time resolution, each channel shifted by its dispersive delay
# (Eq. (3)) and the channels summed, then folded.  Readings:
#   A1  input as the coherent mode: single-pol complex int8 I/Q (C14); the
#       adding of the two telescope halves is therefore absent.
#   A2  channel c of an nchan-point transform is baseband frequency
#       fftfreq(nchan) * bw, i.e. sky f0 + f_c (upper side, as C2); square
#       window, no overlap.
#   A3  delays by the constant of C1, referred to f0 like the coherent
#       outputs: dt_c = (DM / 2.41e-4) (f_c^-2 - f0^-2) s, rounded to the
#       nearest integrated sample: d_c = floor(dt_c / t_s + 1/2),
#       t_s = nchan * nint / fs.
#   A4  output m (m >= 0) is the sum over c of channel c at integrated
#       sample m + d_c - d_min; only outputs every channel covers exist.
#       Its time (that of its f0 channel, d = 0) is (m - d_min) t_s from the
#       stream start, and its fold phase x = (m - d_min) nchan nint / (P fs)
#       (float64), binned as C9.
# --------------------------------------------------------------------------
def aid_filterbank(iq, nchan, nint):
    """Integrated power spectra F[t, c] (float64): the sum over nint
    consecutive spectra of |FFT_nchan(block)|^2, blocks back to back."""
    x = unpack(iq)
    t = x.size // (nchan * nint)
    blocks = x[:t * nchan * nint].reshape(t * nint, nchan)
    p = np.abs(sfft.fft(blocks, axis=1)) ** 2
    return p.reshape(t, nint, nchan).sum(axis=1)


def aid_delays(f0_mhz, bw_mhz, dm, nchan, nint):
    """Per-channel delay in integrated samples (reading A3) and t_s."""
    f = f0_mhz + sfft.fftfreq(nchan, d=1.0 / bw_mhz)
    ts = nchan * nint / (bw_mhz * 1e6)
    dt = DM_CONST_S * dm * (1.0 / (f * f) - 1.0 / (f0_mhz * f0_mhz))
    return np.floor(dt / ts + 0.5).astype(np.int64), ts


def aid_dedisperse(F, d):
    """D[m] = sum_c F[m + d_c - d_min, c] over the outputs every channel
    covers (reading A4)."""
    dd = d - d.min()
    t_out = F.shape[0] - int(dd.max())
    if t_out <= 0:
        return np.zeros(0)
    D = np.zeros(t_out)
    for c in range(F.shape[1]):
        D += F[dd[c]:dd[c] + t_out, c]
    return D


def aid_run(iq, f0_mhz, bw_mhz, dm, nchan, nint, nbins, period_s):
    """The AID path over one stream: dedispersed series and its folded
    profile (mean per bin)."""
    F = aid_filterbank(iq, nchan, nint)
    d, ts = aid_delays(f0_mhz, bw_mhz, dm, nchan, nint)
    D = aid_dedisperse(F, d)
    dmin = int(d.min())
    m = np.arange(D.size)
    inv_pfs = 1.0 / (period_s * bw_mhz * 1e6)
    x = (m - dmin).astype(np.float64) * float(nchan * nint) * inv_pfs
    b = np.minimum(np.floor((x - np.floor(x)) * nbins).astype(np.int64), nbins - 1)
    sums = np.bincount(b, weights=D, minlength=nbins)
    cnts = np.bincount(b, minlength=nbins)
    prof = np.where(cnts > 0, sums / np.maximum(cnts, 1), 0.0)
    return dict(series=D, profile=prof, counts=cnts, delays=d, d_min=dmin, t_s=ts, filterbank=F)


# --------------------------------------------------------------------------
# The paper's own input path: two telescope halves, real-sampled (Sec. 2:
# two 8-bit ADC channels, the 16 MHz band Nyquist-sampled at 32 Msps each),
# added in phase (the AIP kernel, Sec. 3.7) and dedispersed through a
# real-to-complex transform.  Readings:
#   R1  input bytes interleave the channels, A0 B0 A1 B1 ...; adding in
#       phase is the plain sum x[n] = A[n] + B[n] (the halves arrive
#       phased; the paper gives no further step).
#   R2  x is sampled at fs_r = 2 bw; real-FFT bin k (0 <= k <= N_r/2) is
#       baseband fb = k fs_r / N_r.  Upper sideband: sky f0 - bw/2 + fb;
#       lower sideband (the paper's 38 MHz mix of a 22-38 MHz IF): sky
#       f0 + bw/2 - fb.  With f the offset from f0, bin k is multiplied by
#       exp(-2 pi i turns(f)) (upper) or exp(+2 pi i turns(f)) (lower: the
#       band is mirrored, so its phase is conjugated), times the taper of
#       C4; the DC and Nyquist bins keep only the real part of that factor
#       (the inverse real transform has no imaginary part there).
#   R3  geometry in complex-equivalent units: a block of N_r = 2 N real
#       samples, with N, n_front and hop of the complex plan of the same
#       bandwidth (plan_geometry(f0, bw, dm, N)), doubled: the real-rate
#       smear never exceeds twice the complex-rate one.
#   R4  detection y[n]^2 of the real dedispersed voltage; series sums of
#       decim real samples; fold phase of real output r is
#       (r + 2 n_front) / (P fs_r).
# --------------------------------------------------------------------------
def aip(raw):
    """Adding in phase (R1): interleaved int8 A0 B0 A1 B1 ... -> A + B, float64."""
    raw = np.asarray(raw)
    return raw[0::2].astype(np.float64) + raw[1::2].astype(np.float64)


def real_chirp(nfft_r, f0_mhz, bw_mhz, dm, sideband, taper_alpha=0.0):
    """Multiplier of the real-FFT bins 0..nfft_r/2 (reading R2)."""
    fb = np.arange(nfft_r // 2 + 1) * (2.0 * bw_mhz / nfft_r)
    if sideband == "usb":
        f = fb - bw_mhz / 2
        m = np.exp(-2j * np.pi * chirp_turns(f, f0_mhz, dm))
    elif sideband == "lsb":
        f = bw_mhz / 2 - fb
        m = np.exp(+2j * np.pi * chirp_turns(f, f0_mhz, dm))
    else:
        raise ValueError("sideband must be 'usb' or 'lsb'")
    m = m * taper(f, bw_mhz, taper_alpha)
    m[0] = m[0].real
    m[-1] = m[-1].real
    return m


def run_real(raw, f0_mhz, bw_mhz, dm, nfft, nbins, period_s, sideband="lsb",
             subint_nsamp=0, decim=32, taper_alpha=0.0, keep_power=False):
    """The real two-channel path (R1-R4) over one stream: blocks of 2*nfft
    real samples, every fully covered block; subint_nsamp and decim in real
    samples.  Same result dict as `run`, with outputs counted in real
    samples."""
    g = plan_geometry(f0_mhz, bw_mhz, dm, nfft)
    n_r, hop_r, nf_r = 2 * nfft, 2 * g["hop"], 2 * g["n_front"]
    fs_r = 2.0 * bw_mhz * 1e6
    x = aip(raw)
    nb = n_blocks(x.size, n_r, hop_r)
    n_out = nb * hop_r
    m = real_chirp(n_r, f0_mhz, bw_mhz, dm, sideband, taper_alpha)
    p = np.empty(n_out)
    for b in range(nb):
        y = sfft.irfft(sfft.rfft(x[b * hop_r:b * hop_r + n_r]) * m, n=n_r)
        p[b * hop_r:(b + 1) * hop_r] = y[nf_r:nf_r + hop_r] ** 2
    series = decimate(p, decim)
    ns_total = (max(n_out - 1, 0) // subint_nsamp + 1) if (subint_nsamp > 0 and n_out) else (1 if n_out else 0)
    sums = np.zeros((ns_total, nbins))
    cnts = np.zeros((ns_total, nbins), dtype=np.int64)
    if n_out:
        s, c, s0 = fold(p, 0, nf_r, period_s, fs_r, nbins, subint_nsamp)
        sums[s0:s0 + s.shape[0]] += s
        cnts[s0:s0 + c.shape[0]] += c
    complete = (n_out // subint_nsamp) if subint_nsamp > 0 else 0
    return dict(geometry=dict(g, n_r=n_r, hop_r=hop_r, n_front_r=nf_r, fs_r=fs_r), n_out=n_out,
                series=series, sums=sums, cnts=cnts, profiles=profiles_from(sums, cnts),
                complete=complete, power=p if keep_power else None)


def disperse_real(x, f0_mhz, bw_mhz, dm, nfft_r, sideband="lsb"):
    """The real-path forward model: the ISM response applied to a real
    stream by overlap-save (the conjugate of real_chirp's phase); x covers
    2*pad_lo samples before and 2*pad_hi after the part kept."""
    pad_lo, pad_hi = disperse_pads(f0_mhz, bw_mhz, dm)
    lo, hi = 2 * pad_lo, 2 * pad_hi
    hop = nfft_r - lo - hi
    if hop <= 0:
        raise ValueError("nfft too short to disperse")
    n_keep = x.size - lo - hi
    h = np.conj(real_chirp(nfft_r, f0_mhz, bw_mhz, dm, sideband))
    nb = -(-n_keep // hop)
    xp = np.zeros(nb * hop + lo + hi + nfft_r)
    xp[:x.size] = x
    out = np.empty(nb * hop)
    for b in range(nb):
        y = sfft.irfft(sfft.rfft(xp[b * hop:b * hop + nfft_r]) * h, n=nfft_r)
        out[b * hop:(b + 1) * hop] = y[lo:lo + hop]
    return out[:n_keep]
