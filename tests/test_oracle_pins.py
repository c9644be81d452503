"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks it against a value
printed in the paper (tests/golden/paper_values.json), a closed form, an
invariant, a brute-force O(N^2) evaluation or exact integer arithmetic.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

F0, BW = 326.5, 16.0


# --------------------------------------------------------------- constants
def test_dispersion_constant_matches_eq3_and_eq4(golden):
    # Eq. (3): 4.15e6 ms == 4.15e3 s per unit DM per MHz^-2
    assert abs(O.DM_CONST_S / (golden["eq3_coefficient_ms"]["value"] * 1e-3) - 1) < 1e-3
    # Eq. (4): phase 8.3e3 * pi * DM f^2/(f0^2 (f+f0)); with the missing 1e6
    # (MHz -> Hz) that is 2 pi DM_CONST_TURNS
    assert abs(2 * O.DM_CONST_TURNS / (golden["eq4_coefficient"]["value"] * 1e6) - 1) < 1e-3
    # Eq. (1) constant is the one used
    assert O.DM_CONST_S == 1.0 / golden["eq1_constant"]["value"]


def test_eq2_smear_across_band_matches_exact_delay(golden):
    g = O.plan_geometry(F0, BW, 1.0, 1 << 18)
    exact_ms = (g["delta_lo"] + g["delta_hi"]) * 1e3
    eq2 = O.residual_smear_ms(BW, F0, 1.0)
    assert abs(eq2 / exact_ms - 1) < 2e-3            # 3.815 vs 3.819 ms
    assert abs(exact_ms - 3.8195) < 1e-3


def test_1024_channel_smear_printed_in_paper(golden):
    # Sec. 3.4: 1024 channels over 16 MHz leave ~3.8 us per unit DM
    dfc = BW / 1024
    exact_us = O.dispersion_delay_s(F0 - dfc / 2, F0 + dfc / 2, 1.0) * 1e6
    eq2_us = O.residual_smear_ms(dfc, F0, 1.0) * 1e3
    printed = golden["smear_1024ch_us_per_dm"]["value"]
    assert abs(exact_us / printed - 1) < 0.03
    assert abs(eq2_us / printed - 1) < 0.03


def test_base_and_integrated_resolution(golden):
    g = O.plan_geometry(F0, BW, 1.0, 1 << 18)
    assert 1.0 / g["fs"] == pytest.approx(golden["base_resolution_s"]["value"], rel=1e-12)
    assert 16 / g["fs"] == pytest.approx(golden["integrated_resolution_s"]["value"], rel=1e-12)


def test_eq1_reading_is_documented(golden):
    # Reading C12: N = 2 smear / ts; at DM 130 this gives 2^23.9, not the
    # paper's 2^27 (documented discrepancy, not a requirement of the build).
    n = O.fft_length_eq1(F0 + BW / 2, BW, 130.0, golden["base_resolution_s"]["value"])
    assert 23.8 < math.log2(n) < 24.0


# ------------------------------------------------------------------- chirp
@pytest.mark.parametrize("dm", [0.0, 1.0, 50.0, 200.0])
def test_chirp_unit_modulus(dm):
    C = O.dedispersion_chirp(1 << 16, F0, BW, dm)
    H = O.ism_response(1 << 16, F0, BW, dm)
    assert np.max(np.abs(np.abs(C) - 1)) < 1e-15
    assert np.max(np.abs(C * np.conj(C) - 1)) < 1e-15
    assert np.max(np.abs(H * C - 1)) < 1e-14
    assert C[0] == 1.0
    if dm == 0.0:
        assert np.all(C == 1.0)


@pytest.mark.parametrize("dm", [1.0, 50.0, 200.0])
def test_group_delay_is_cold_plasma_delay(dm):
    """-d(turns)/df of the ISM response is the delay of Eq. (3)'s form."""
    f = np.linspace(-BW / 2 * 0.999, BW / 2 * 0.999, 257)
    h = 1e-4
    slope = (O.chirp_turns(f + h, F0, dm) - O.chirp_turns(f - h, F0, dm)) / (2 * h)  # turns/MHz = us
    # H = exp(+2 pi i turns), numpy convention: a delay tau multiplies the
    # spectrum by exp(-2 pi i f tau) -> tau = -d(phase)/d(2 pi f)
    tau_s = -slope * 1e-6
    want = O.dispersion_delay_s(F0 + f, F0, dm)
    # lower frequencies later (positive), upper earlier
    assert np.all(want[f < 0] > 0) and np.all(want[f > 0] < 0)
    np.testing.assert_allclose(tau_s, want, rtol=1e-7, atol=1e-12)


def test_dispersed_impulse_arrives_at_subband_delays():
    """A dispersed impulse: in each of 16 sub-bands the energy centroid lies
    at the cold-plasma delay of that sub-band's centre."""
    dm = 1.0
    fs = BW * 1e6
    pad_lo, pad_hi = O.disperse_pads(F0, BW, dm)
    L = 1 << 17
    t0 = 40000
    z = np.zeros(pad_lo + L + pad_hi, dtype=np.complex128)
    z[pad_lo + t0] = 1.0
    out = O.disperse(z, F0, BW, dm, 1 << 18)
    S = np.fft.fft(out)
    fr = np.fft.fftfreq(out.size, 1.0 / BW)
    edges = np.linspace(-BW / 2, BW / 2, 17)
    for lo, hi in zip(edges[:-1], edges[1:]):
        mask = (fr >= lo) & (fr < hi)
        sub = np.fft.ifft(np.where(mask, S, 0))
        w = np.abs(sub) ** 2
        t = np.arange(out.size)
        centroid = (w * t).sum() / w.sum()
        fc = 0.5 * (lo + hi)
        want = t0 + O.dispersion_delay_s(F0 + fc, F0, dm) * fs
        sub_smear = (O.dispersion_delay_s(F0 + lo, F0, dm) - O.dispersion_delay_s(F0 + hi, F0, dm)) * fs
        assert abs(centroid - want) < 0.05 * sub_smear + 3, (lo, hi, centroid, want)


# --------------------------------------------------------------------- FFT
def _brute_dft(x, sign):
    n = x.size
    k = np.arange(n)
    W = np.exp(sign * 2j * np.pi * np.outer(k, k) / n)
    return W @ x


@pytest.mark.parametrize("n", [8, 16, 64])
def test_block_transform_is_brute_force_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    C = np.exp(2j * np.pi * rng.random(n))
    got = O.dedisperse_block(x, C, 0, n)
    want = _brute_dft(_brute_dft(x, -1) * C, +1) / n
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(x).max())


def test_parseval_and_all_pass_energy():
    rng = np.random.default_rng(3)
    n = 1 << 14
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = np.fft.fft(x)
    assert abs(np.sum(np.abs(X) ** 2) / n / np.sum(np.abs(x) ** 2) - 1) < 1e-12
    C = O.dedispersion_chirp(n, F0, BW, 3.0)
    y = O.dedisperse_block(x, C, 0, n)
    assert abs(np.sum(np.abs(y) ** 2) / np.sum(np.abs(x) ** 2) - 1) < 1e-12


def test_overlap_save_equals_brute_circular_convolution():
    """Valid outputs of every block equal the O(N^2) circular convolution of
    that block with h = IDFT(H^-1), and land at outputs m = b*hop + j."""
    n, dm = 256, 0.001
    g = O.plan_geometry(F0, BW, dm, n)
    assert g["discard"] == 64 and g["hop"] == 192
    rng = np.random.default_rng(7)
    iq = rng.integers(-128, 128, size=2 * (n + 3 * g["hop"])).astype(np.int8)
    x = iq[0::2].astype(np.float64) + 1j * iq[1::2]
    C = O.dedispersion_chirp(n, F0, BW, dm)
    h = _brute_dft(C, +1) / n
    y, m0 = O.dedisperse(O.unpack(iq), F0, BW, dm, n)
    assert m0 == 0 and y.size == 4 * g["hop"]
    idx = np.arange(n)
    for b in range(4):
        xb = x[b * g["hop"]:b * g["hop"] + n]
        conv = np.array([np.sum(xb * h[(i - idx) % n]) for i in range(n)])
        want = conv[g["n_front"]:g["n_front"] + g["hop"]]
        np.testing.assert_allclose(y[b * g["hop"]:(b + 1) * g["hop"]], want, rtol=0, atol=1e-9)


# -------------------------------------------------------------------- fold
def _brute_fold(p, m0, n_front, period_s, fs, nbins, S):
    inv = 1.0 / (period_s * fs)
    sums, cnts = {}, {}
    for i, v in enumerate(p):
        m = m0 + i
        x = float(m + n_front) * inv
        b = min(int(math.floor((x - math.floor(x)) * nbins)), nbins - 1)
        s = m // S if S > 0 else 0
        sums[(s, b)] = sums.get((s, b), 0.0) + float(v)
        cnts[(s, b)] = cnts.get((s, b), 0) + 1
    return sums, cnts


@pytest.mark.parametrize("S", [0, 37, 1000])
def test_fold_matches_python_loop(S):
    rng = np.random.default_rng(11)
    p = rng.random(3001) * 100
    m0, nf, nbins, period, fs = 777, 123, 13, 1.234e-5, 16e6
    sums, cnts, s0 = O.fold(p, m0, nf, period, fs, nbins, S)
    bs, bc = _brute_fold(p, m0, nf, period, fs, nbins, S)
    for s in range(sums.shape[0]):
        for b in range(nbins):
            assert cnts[s, b] == bc.get((s0 + s, b), 0)
            assert sums[s, b] == pytest.approx(bs.get((s0 + s, b), 0.0), rel=1e-12, abs=1e-9)
    assert cnts.sum() == p.size


def test_fold_bins_integer_period_exact_counts():
    """P fs = 1425600 samples (P = 0.0891 s at 16 Msps): the bin of sample n
    is floor(256 n / 1425600) exactly, except at exact bin edges where the
    float64 rounding of 1/(P fs) may put it one bin lower."""
    nbins, P, fs = 256, 0.0891, 16e6
    n = np.arange(1425600, dtype=np.int64)
    b = O.fold_bins(n, 0, P, fs, nbins)
    exact = (n * nbins) // 1425600
    tie = (n * nbins) % 1425600 == 0
    assert np.all(b[~tie] == exact[~tie])
    assert np.all((b[tie] == exact[tie]) | (b[tie] == exact[tie] - 1))
    counts = np.bincount(b, minlength=nbins)
    ex_counts = np.bincount(exact, minlength=nbins)
    assert counts.sum() == n.size
    assert np.max(np.abs(counts - ex_counts)) <= 1
    assert set(np.unique(ex_counts)) <= {5568, 5569}


def test_dm0_reduces_to_plain_fold_of_power():
    """DM = 0: H^-1 = 1, no discard, so the method is |x|^2 folded directly."""
    rng = np.random.default_rng(5)
    n = 1024
    iq = rng.integers(-128, 128, size=2 * 3 * n).astype(np.int8)
    r = O.run(iq, F0, BW, 0.0, n, nbins=7, period_s=2.3e-5, subint_nsamp=500,
              decim=4, keep_power=True)
    x = iq[0::2].astype(np.float64) + 1j * iq[1::2]
    pw = np.abs(x) ** 2
    assert r["geometry"]["discard"] == 0 and r["n_out"] == 3 * n
    np.testing.assert_allclose(r["power"], pw, rtol=1e-12, atol=1e-9)
    bs, bc = _brute_fold(pw, 0, 0, 2.3e-5, 16e6, 7, 500)
    for (s, b), v in bs.items():
        assert r["cnts"][s, b] == bc[(s, b)]
        assert r["sums"][s, b] == pytest.approx(v, rel=1e-10)
    np.testing.assert_allclose(r["series"], pw.reshape(-1, 4).sum(1), rtol=1e-10)


def test_series_fold_and_count_invariants():
    rng = np.random.default_rng(9)
    n = 1 << 12
    iq = rng.integers(-60, 60, size=2 * 5 * n).astype(np.int8)
    r = O.run(iq, F0, BW, 0.05, n, nbins=32, period_s=1.1e-4, subint_nsamp=3000,
              decim=16, keep_power=True)
    g = r["geometry"]
    assert r["n_out"] == O.n_blocks(5 * n, n, g["hop"]) * g["hop"]
    assert r["cnts"].sum() == r["n_out"]
    assert r["series"].sum() == pytest.approx(r["power"].sum(), rel=1e-12)
    assert r["sums"].sum() == pytest.approx(r["power"].sum(), rel=1e-12)
    assert r["complete"] == r["n_out"] // 3000


# ---------------------------------------------------------------- geometry
def test_geometry_of_stated_workloads():
    g0 = O.plan_geometry(F0, BW, 1.0, 1 << 18)
    assert (g0["n_front"], g0["discard"], g0["hop"]) == (29434, 1 << 16, 196608)
    g1 = O.plan_geometry(F0, BW, 50.0, 1 << 23)
    assert (g1["n_front"], g1["discard"], g1["hop"]) == (1471655, 1 << 22, 1 << 22)
    assert O.n_blocks(960_000_000, 1 << 23, g1["hop"]) == 227
    g4 = O.plan_geometry(F0, BW, 200.0, 1 << 24)
    assert (g4["discard"], g4["hop"]) == (12222368, 4554848)
    gz = O.plan_geometry(F0, BW, 0.0, 1 << 10)
    assert (gz["n_front"], gz["discard"], gz["hop"]) == (0, 0, 1 << 10)
    with pytest.raises(ValueError):
        O.plan_geometry(F0, BW, 200.0, 1 << 20)


# ----------------------------------------------------- end to end (config 0)
def _config0_stream(seed=1, nsamp=8_000_000, dm=1.0):
    fs = BW * 1e6
    pad_lo, pad_hi = O.disperse_pads(F0, BW, dm)
    z = synth.pulsed_noise(seed, pad_lo + nsamp + pad_hi, first_index=-pad_lo, fs_hz=fs)
    return synth.quantize_int8(O.disperse(z, F0, BW, dm, 1 << 20))


@pytest.fixture(scope="module")
def config0_iq():
    return _config0_stream()


def test_pulse_recovered_at_true_dm(config0_iq):
    """Dedispersing the config-0 stream recovers the injected pulse: each bin
    matches 800 (1 + 3 g_bin) + 1/6 within its own statistics."""
    nbins, P = 256, synth.PERIOD_S
    r = O.run(config0_iq, F0, BW, 1.0, 1 << 18, nbins, P, subint_nsamp=0, decim=16)
    g = r["geometry"]
    assert r["n_out"] == 7_864_320
    m = np.arange(r["n_out"], dtype=np.int64)
    b = O.fold_bins(m, g["n_front"], P, g["fs"], nbins)
    shape = synth.pulse_power_shape(m + g["n_front"], g["fs"])
    mean_i = 2 * synth.SIGMA ** 2 * shape + 1.0 / 6.0
    cnt = np.bincount(b, minlength=nbins)
    want = np.bincount(b, weights=mean_i, minlength=nbins) / cnt
    sd = np.sqrt(np.bincount(b, weights=mean_i ** 2, minlength=nbins)) / cnt
    z = (r["profiles"][0] - want) / sd
    assert np.max(np.abs(z)) < 5.5, np.argmax(np.abs(z))
    chi2 = np.mean(z ** 2)
    assert 0.7 < chi2 < 1.4
    assert abs(int(np.argmax(r["profiles"][0])) - nbins // 2) <= 1
    np.testing.assert_array_equal(r["cnts"][0], cnt)


def test_dm0_processing_leaves_the_dispersion_smear(config0_iq):
    """Folding the same stream without dedispersion smears the pulse over the
    ~3.8 ms band delay: lower peak, wider profile (the synthetic analogue of
    the coherent vs incoherent comparison of Sec. 4)."""
    nbins, P = 256, synth.PERIOD_S
    good = O.run(config0_iq, F0, BW, 1.0, 1 << 18, nbins, P)["profiles"][0]
    raw = O.run(config0_iq, F0, BW, 0.0, 1 << 18, nbins, P)["profiles"][0]
    base = 800.17
    pk_good, pk_raw = good.max() - base, raw.max() - base
    assert pk_raw < 0.6 * pk_good
    w_good = np.sum(good - base > pk_good / 2)
    w_raw = np.sum(raw - base > pk_raw / 2)
    assert w_raw > 2.5 * w_good


# ---------------------------------------------------------------- taper (C4)
def test_taper_window_shape():
    """Tukey window over [-bw/2, bw/2]: 1 in the flat part, 1/2 at the middle
    of each edge, 0 at the band edge, even in f, non-increasing in |f|;
    alpha = 0 is the unit taper."""
    bw, alpha = 16.0, 0.3
    f = np.linspace(-8.0, 8.0, 4001)
    w = O.taper(f, bw, alpha)
    assert np.all(O.taper(f, bw, 0.0) == 1.0)
    assert O.taper(np.array([0.0]), bw, alpha)[0] == 1.0
    assert np.allclose(O.taper(np.array([-8.0, 8.0]), bw, alpha), 0.0, atol=1e-15)
    mid = (1 - alpha / 2) * bw / 2
    assert np.allclose(O.taper(np.array([-mid, mid]), bw, alpha), 0.5)
    assert np.allclose(w, w[::-1])
    half = w[f >= 0]
    assert np.all(np.diff(half) <= 1e-15) and np.all((w >= 0) & (w <= 1))


def test_full_band_taper_is_three_tap_filter():
    """alpha = 1 makes the window 1/2 + cos(2 pi k / N)/2 on the FFT grid,
    whose inverse transform is the three taps 1/4, 1/2, 1/4: at DM 0 an
    impulse comes out as exactly that, and a white stream keeps 3/8 of its
    power (sum of squared taps)."""
    n = 1 << 10
    x = np.zeros(n, dtype=np.complex128)
    x[300] = 1.0
    y, _ = O.dedisperse(x, 326.5, 16.0, 0.0, n, taper_alpha=1.0)
    want = np.zeros(n)
    want[299:302] = [0.25, 0.5, 0.25]
    assert np.allclose(y.real, want, atol=1e-12) and np.allclose(y.imag, 0, atol=1e-12)
    rng = np.random.default_rng(3)
    z = rng.normal(size=n) + 1j * rng.normal(size=n)
    y, _ = O.dedisperse(z, 326.5, 16.0, 0.0, n, taper_alpha=1.0)
    brute = 0.25 * np.roll(z, 1) + 0.5 * z + 0.25 * np.roll(z, -1)
    assert np.allclose(y, brute, atol=1e-12)


def test_unit_taper_is_the_default():
    iq = synth.white_stream_int8(8, 20000)
    a = O.run(iq, 326.5, 16.0, 0.01, 1 << 12, 32, 1e-3)
    b = O.run(iq, 326.5, 16.0, 0.01, 1 << 12, 32, 1e-3, taper_alpha=0.0)
    assert np.array_equal(a["profiles"], b["profiles"]) and np.array_equal(a["series"], b["series"])


# ------------------------------------------------- AID (incoherent) mode
def test_aid_filterbank_tone_and_parseval():
    """A complex tone on channel 37 puts all of a block's power there
    (nchan^2 A^2 per block), and every integrated spectrum sums to nchan
    times the block energy (Parseval)."""
    nchan, nint = 64, 3
    n = np.arange(nchan * nint * 5)
    x = 2.0 * np.exp(2j * np.pi * 37 * n / nchan)
    iq = np.empty(2 * n.size)
    iq[0::2], iq[1::2] = x.real, x.imag
    F = O.aid_filterbank(iq, nchan, nint)
    assert F.shape == (5, nchan)
    assert np.allclose(F[:, 37], nint * nchan ** 2 * 4.0)
    assert np.allclose(np.delete(F, 37, axis=1), 0, atol=1e-6)
    rng = np.random.default_rng(4)
    z = rng.integers(-128, 128, size=2 * nchan * nint * 7).astype(np.int8)
    F = O.aid_filterbank(z, nchan, nint)
    e = (z.astype(np.float64) ** 2).reshape(7, nint * nchan * 2).sum(axis=1)
    assert np.allclose(F.sum(axis=1), nchan * e)


def test_aid_delays_follow_eq3():
    """Delays referred to f0: zero at f0, larger (later) below it, the band
    edge at (DM/2.41e-4)(f^-2 - f0^-2) s; ~4.15e6 ms MHz^2 as printed in Eq. (3)."""
    f0, bw, dm, nchan, nint = 326.5, 16.0, 50.0, 1024, 4
    d, ts = O.aid_delays(f0, bw, dm, nchan, nint)
    assert ts == nchan * nint / 16e6 and d[0] == 0
    f = f0 + np.fft.fftfreq(nchan, 1 / bw)
    order = np.argsort(f)
    assert np.all(np.diff(d[order]) <= 0)
    lo = order[0]
    want = 4.15e6 * (f[lo] ** -2 - f0 ** -2) * dm * 1e-3 / ts
    assert abs(d[lo] - want) / want < 2e-3


def test_aid_dedisperse_brute_force():
    """Tiny case against explicit loops."""
    rng = np.random.default_rng(5)
    F = rng.normal(size=(40, 6))
    d = np.array([0, 3, -2, 5, 1, -2])
    D = O.aid_dedisperse(F, d)
    dd = d - d.min()
    t_out = 40 - dd.max()
    want = [sum(F[m + dd[c], c] for c in range(6)) for m in range(t_out)]
    assert np.allclose(D, want)


def test_aid_recovers_dispersed_pulse():
    """A pulse dispersed at DM 5 folds sharply at phase 0.5 with the AID
    path at DM 5, and smeared at DM 0 (64 channels of 250 kHz)."""
    fs, period = 16e6, 0.02
    pad_lo, pad_hi = O.disperse_pads(326.5, 16.0, 5.0)
    z = synth.pulsed_noise(12, pad_lo + 4_000_000 + pad_hi, first_index=-pad_lo, fs_hz=fs,
                           period_s=period, fwhm_s=2e-4, peak=20.0)
    iq = synth.quantize_int8(O.disperse(z, 326.5, 16.0, 5.0, 1 << 21))
    r5 = O.aid_run(iq, 326.5, 16.0, 5.0, 64, 8, 64, period)
    r0 = O.aid_run(iq, 326.5, 16.0, 0.0, 64, 8, 64, period)
    p5, p0 = r5["profile"], r0["profile"]
    assert abs(int(np.argmax(p5)) - 32) <= 1
    snr = lambda p: (p.max() - np.median(p)) / p[np.abs(np.arange(64) - 32) > 8].std()
    assert snr(p5) > 3 * snr(p0), (snr(p5), snr(p0))


# --------------------------------------- real two-channel input path (AIP)
def _two_channel(x, seed, noise=0.0):
    """Interleave x (+ independent noise per channel) as int8 A0 B0 A1 ..."""
    rng = np.random.default_rng(seed)
    a = np.clip(np.rint(x / 2 + noise * rng.normal(size=x.size)), -128, 127)
    b = np.clip(np.rint(x / 2 + noise * rng.normal(size=x.size)), -128, 127)
    raw = np.empty(2 * x.size, dtype=np.int8)
    raw[0::2], raw[1::2] = a, b
    return raw


def test_aip_adds_the_halves():
    raw = np.array([3, -1, 127, -128, 0, 5], dtype=np.int8)
    assert np.array_equal(O.aip(raw), [2.0, -1.0, 5.0])


def test_real_path_is_identity_at_dm0():
    """Unit taper and DM 0: the multiplier is 1 on every bin, so the
    dedispersed voltage is the added-in-phase input and the series its
    decimated square."""
    rng = np.random.default_rng(6)
    raw = rng.integers(-128, 128, size=2 * 40000).astype(np.int8)
    r = O.run_real(raw, 326.5, 16.0, 0.0, 1 << 12, 16, 1e-3, decim=32, keep_power=True)
    x = O.aip(raw)
    assert np.allclose(r["power"], x[:r["n_out"]] ** 2, rtol=1e-9, atol=1e-6)
    assert np.allclose(r["series"], O.decimate(x[:r["n_out"]] ** 2, 32))


def test_real_dispersed_tone_delays_follow_the_sideband():
    """A real tone burst at baseband fb, dispersed by the real forward model,
    arrives with the cold-plasma delay of its SKY frequency: f0 + bw/2 - fb
    for the lower sideband, f0 - bw/2 + fb for the upper one (delays
    referred to f0, later below it)."""
    fs_r, n = 32e6, 1 << 20
    t = np.arange(n)
    for sideband, fb in (("lsb", 3.0), ("lsb", 13.0), ("usb", 3.0)):
        env = np.exp(-0.5 * ((t - n // 2) / 400.0) ** 2)
        x = env * np.cos(2 * np.pi * fb * 1e6 * t / fs_r)
        pad_lo, pad_hi = O.disperse_pads(326.5, 16.0, 2.0)
        xp = np.concatenate([np.zeros(2 * pad_lo), x, np.zeros(2 * pad_hi)])
        y = O.disperse_real(xp, 326.5, 16.0, 2.0, 1 << 22, sideband)
        # arrival = centroid of the detected burst
        p = y ** 2
        arrival = (np.sum(p * t) / np.sum(p) - n // 2) / fs_r
        f_sky = 326.5 + 8.0 - fb if sideband == "lsb" else 326.5 - 8.0 + fb
        want = O.dispersion_delay_s(f_sky, 326.5, 2.0)
        assert abs(arrival - want) < 2e-6, (sideband, fb, arrival, want)


def test_real_path_recovers_a_pulse_lsb():
    """Pulsed real noise in both halves, dispersed (lower sideband) at DM 2,
    added in phase and dedispersed: the pulse is sharp at phase 0.5 and
    the dedispersed power matches the undispersed one (|H| = 1)."""
    fs_r, period, n = 32e6, 0.01, 2_000_000
    pad_lo, pad_hi = O.disperse_pads(326.5, 16.0, 2.0)
    rng = np.random.default_rng(7)
    tt = (np.arange(-2 * pad_lo, n + 2 * pad_hi)) / fs_r
    ph = (tt / period) % 1.0
    g = 1.0 + 8.0 * np.exp(-0.5 * ((ph - 0.5) / (1e-4 / period)) ** 2)
    s = rng.normal(size=tt.size) * 20.0 * np.sqrt(g)
    # band-limit to (0, bw) with a real FFT so both sidebands see the same band
    x = O.disperse_real(s, 326.5, 16.0, 2.0, 1 << 23, "lsb")
    raw = _two_channel(x, 8, noise=5.0)
    r = O.run_real(raw, 326.5, 16.0, 2.0, 1 << 19, 64, period, sideband="lsb", decim=32)
    prof = r["profiles"][0]
    assert abs(int(np.argmax(prof)) - 32) <= 1
    r0 = O.run_real(raw, 326.5, 16.0, 2.0, 1 << 19, 64, period, sideband="usb", decim=32)
    assert prof.max() / np.median(prof) > 1.5 * r0["profiles"][0].max() / np.median(r0["profiles"][0])


# ----------------------------------------- negative control: phase precision
def test_float32_chirp_phase_is_far_outside_the_profile_bound():
    """The chirp phase reaches about 3.7e5 turns at the band edge at DM 50,
    where a float32 phase (turns evaluated in float32, not reduced in
    float64) is off by hundredths of a turn: a dedispersion with it misses
    the float64 result by far more than the 1e-4 profile bound, which is why
    the phase is evaluated in float64 everywhere.  (The planted float32 phase
    lives in this test only.)"""
    nfft, dm = 1 << 16, 50.0
    f = O.baseband_freqs_mhz(nfft, 16.0)
    turns64 = O.chirp_turns(f, 326.5, dm)
    assert np.abs(turns64).max() > 3e5
    f32 = f.astype(np.float32)
    turns32 = (np.float32(dm) * f32 * f32 / (np.float32(2.41e-10) * np.float32(326.5) ** 2
                                               * (np.float32(326.5) + f32))).astype(np.float64)
    c64 = np.exp(-2j * np.pi * turns64)
    c32 = np.exp(-2j * np.pi * turns32)
    assert np.abs(np.angle(c32 / c64)).max() > 1e-2
    rng = np.random.default_rng(3)
    x = rng.normal(size=nfft) + 1j * rng.normal(size=nfft)
    y64 = np.fft.ifft(np.fft.fft(x) * c64)
    y32 = np.fft.ifft(np.fft.fft(x) * c32)
    p64, p32 = np.abs(y64) ** 2, np.abs(y32) ** 2
    series_err = np.linalg.norm(p32 - p64) / np.linalg.norm(p64)
    assert series_err > 1e-2, series_err
    # the float64 phase reduced mod 1 turn reproduces the unreduced one
    frac = turns64 - np.rint(turns64)
    assert np.allclose(np.exp(-2j * np.pi * frac), c64, atol=1e-9)
