"""Real two-channel input path (channels A and B added in phase, packed
real-to-complex transform, sideband mapping of the filter; Sec. 3.1 and
Sec. 3.2) through the C ABI against the oracle's run_real: profiles and
series element by element, one call and ragged streaming, both sidebands,
the taper, the shortest transform, and the argument checks."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import BW, F0, profile_rel_l2, rel_l2

pytestmark = pytest.mark.gpu

# (profile rel-L2, series rel-L2) per form, as for the complex path
TOL = {"fp32": (1e-6, 1e-5), "mixed_valu": (1e-4, 1e-2)}
# Bound on the per-sample relative error of a detected power (float16
# storage: about 4e-4 measured as the series error at 2 samples per value);
# a profile bin averaging m samples adds 3 EPS / sqrt(m) to its tolerance.
EPS = {"fp32": 1e-6, "mixed_valu": 2e-3}


def profile_tol(precision, n_out, subint, nbins):
    sizes = [subint] * (n_out // subint) + ([n_out % subint] if n_out % subint else []) if subint else [n_out]
    m = max(1.0, min(sizes) / nbins)
    return TOL[precision][0] + 3 * EPS[precision] / np.sqrt(m)


def real_stream(seed, nsamp, dm, period, sideband, nfft_gen=1 << 22):
    """nsamp real samples of pulsed real noise at 2 bw, dispersed for the
    given sideband by the oracle's forward model, as two int8 channels."""
    pad_lo, pad_hi = O.disperse_pads(F0, BW, dm)
    s = synth.pulsed_real_noise(seed, 2 * pad_lo + nsamp + 2 * pad_hi, first_index=-2 * pad_lo,
                                fs_hz=2 * BW * 1e6, period_s=period)
    while 2 * (pad_lo + pad_hi) >= nfft_gen // 2:
        nfft_gen *= 2
    x = O.disperse_real(s, F0, BW, dm, nfft_gen, sideband)
    return synth.two_channel_int8(x, seed + 1000, noise=5.0)


def gpu_real_run(raw, dm, nfft, nbins, period, sideband, precision="fp32", subint=0, decim=32,
                 chunks=None, taper=0.0, max_batch=0):
    """Stream raw (numpy int8 A/B pairs) through a real-input plan in the
    given chunk sizes (real samples, even; one call if None), flush, and
    return (profiles [k, nbins], series) as numpy."""
    import torch
    from paper_1503_01405_amd import Plan
    x = torch.from_numpy(np.ascontiguousarray(raw)).to("cuda")
    nsamp = raw.size // 2
    chunks = [nsamp] if chunks is None else chunks
    plan = Plan(F0, BW, dm, nfft, nbins, period, precision=precision, max_batch=max_batch,
                subint_nsamp=subint, decim=decim, taper_alpha=taper, sideband=sideband)
    profs, sers, pos = [], [], 0
    for c in chunks:
        c = min(c, nsamp - pos)
        pr, se = plan.process(x[2 * pos:2 * (pos + c)])
        profs.append(pr.cpu().numpy())
        sers.append(se.cpu().numpy())
        pos += c
    assert pos == nsamp, (pos, nsamp)
    profs.append(plan.flush(device=x.device).cpu().numpy())
    torch.cuda.synchronize()
    plan.close()
    return np.concatenate(profs, axis=0), np.concatenate(sers)


def oracle_real_run(raw, dm, nfft, nbins, period, sideband, subint=0, decim=32, taper=0.0):
    """Oracle profiles in the library's emission order and the series."""
    r = O.run_real(raw, F0, BW, dm, nfft // 2, nbins, period, sideband=sideband, subint_nsamp=subint,
                   decim=decim, taper_alpha=taper)
    n_out = r["n_out"]
    if subint > 0:
        k = r["complete"]
        rows = [r["profiles"][i] for i in range(k)]
        if n_out > k * subint:
            rows.append(r["profiles"][k])
    else:
        rows = [r["profiles"][0]] if n_out > 0 else []
    return np.array(rows).reshape(-1, nbins), r["series"], r


def check(raw, dm, nfft, nbins, period, sideband, precisions, **kw):
    """Every form in `precisions` against one oracle run."""
    if isinstance(precisions, str):
        precisions = [precisions]
    oprof, oser, r = oracle_real_run(raw, dm, nfft, nbins, period, sideband,
                                     **{k: v for k, v in kw.items() if k in ("subint", "decim", "taper")})
    for precision in precisions:
        prof, ser = gpu_real_run(raw, dm, nfft, nbins, period, sideband, precision=precision, **kw)
        assert prof.shape == oprof.shape and ser.shape == oser.shape, (prof.shape, oprof.shape, ser.shape,
                                                                       oser.shape)
        ep, es = profile_rel_l2(prof, oprof), rel_l2(ser, oser)
        tp = profile_tol(precision, r["n_out"], kw.get("subint", 0), nbins)
        print(f"{sideband} {precision}: n_out={r['n_out']} profile rel-L2 {ep:.3e} (tol {tp:.1e}) "
              f"series rel-L2 {es:.3e}")
        assert ep <= tp and es <= TOL[precision][1], (precision, ep, es)
    return r


@pytest.fixture(scope="module")
def streams():
    # 3,000,002 real samples (about 94 ms at 32 Msps) at DM 3.1, per sideband
    return {sb: real_stream(31 if sb == "lsb" else 32, 3_000_002, 3.1, 3.3e-2, sb) for sb in ("lsb", "usb")}


@pytest.mark.parametrize("sideband", ["lsb", "usb"])
@pytest.mark.parametrize("precision", ["fp32", "mixed_valu"])
def test_real_parity(streams, sideband, precision):
    print(f"case: real {sideband} {precision} nfft=2^20 dm=3.1", flush=True)
    r = check(streams[sideband], 3.1, 1 << 20, 256, 3.3e-2, sideband, precision)
    assert r["n_out"] > 0


def test_real_streaming_subint(streams):
    """Ragged even chunks (input tail carried across calls, 4 bytes per
    packed element), sub-integrations and a finer series."""
    print("case: real lsb streaming subint=400000 decim=8", flush=True)
    chunks = [2, 700_000, 1_048_576, 333_334, 10, 918_080]
    assert sum(chunks) == 3_000_002
    check(streams["lsb"], 3.1, 1 << 20, 128, 3.3e-2, "lsb", ["fp32", "mixed_valu"], subint=400_000, decim=8,
          chunks=chunks, max_batch=2)


@pytest.mark.parametrize("sideband", ["lsb", "usb"])
def test_real_taper(streams, sideband):
    print(f"case: real {sideband} taper 0.3", flush=True)
    check(streams[sideband], 3.1, 1 << 20, 256, 3.3e-2, sideband, ["fp32", "mixed_valu"], taper=0.3)


@pytest.mark.parametrize("nfft,dm", [(1 << 11, 0.003), (1 << 13, 0.02), (1 << 16, 0.3)])
def test_real_short_transforms(nfft, dm):
    """The shortest transforms (packed length 2^10: 32 x 32 four-step)."""
    print(f"case: real short nfft={nfft} dm={dm}", flush=True)
    raw = real_stream(41, 400_006, dm, 1.1e-3, "usb", nfft_gen=1 << 18)
    check(raw, dm, nfft, 64, 1.1e-3, "usb", ["fp32", "mixed_valu"], decim=2)


@pytest.mark.parametrize("nbins", [700, 2000])
def test_real_fine_bins(nbins):
    """Bins about one group of 32 real outputs wide (700) and a third of one
    (2000), with sub-integration edges inside groups' blocks: groups that
    straddle two bins, and groups that span several."""
    print(f"case: real fine bins nbins={nbins}", flush=True)
    raw = real_stream(61, 300_010, 0.02, 7.3e-4, "lsb", nfft_gen=1 << 18)
    check(raw, 0.02, 1 << 13, nbins, 7.3e-4, "lsb", ["fp32", "mixed_valu"], subint=50_002, decim=4)


@pytest.mark.parametrize("nfft,dm,sideband", [(1 << 22, 3.1, "lsb"), (1 << 23, 10.0, "usb"), (1 << 24, 20.0, "lsb"),
                                              (1 << 25, 1.0, "usb")])
def test_real_long_rows(nfft, dm, sideband):
    """Rows of 2^11 to 2^13 (one fused middle pass; 2^13 is the 60 s
    workload's shape) and 2^14 (forward rows, split, inverse rows), over a
    little more than two blocks."""
    import oracle as O
    g = O.plan_geometry(F0, BW, dm, nfft // 2)
    nsamp = nfft + 2 * g["hop"] + 1002
    print(f"case: real long rows nfft=2^{nfft.bit_length() - 1} dm={dm} {sideband} nsamp={nsamp}", flush=True)
    raw = real_stream(51, nsamp, dm, 0.0891, sideband)
    r = check(raw, dm, nfft, 1024, 0.0891, sideband, ["fp32", "mixed_valu"], decim=32)
    assert r["n_out"] == 4 * g["hop"]


def test_real_api():
    """Units reported in real samples, and the argument checks."""
    import torch
    import paper_1503_01405_amd as P
    print("case: real api", flush=True)
    h = P.pond_real_plan_create(F0, BW, 3.1, 1 << 20, 64, 3.3e-2, P.POND_FP32, 0, "usb")
    hc = P.pond_plan_create(F0, BW, 3.1, 1 << 19, 64, 3.3e-2)
    try:
        info, ic = P.pond_plan_query(h), P.pond_plan_query(hc)
        assert info["input_kind"] == P.POND_INPUT_REAL_USB and ic["input_kind"] == P.POND_INPUT_COMPLEX
        assert info["nfft"] == 1 << 20 and info["n1"] * info["n2"] == 1 << 19
        for k in ("n_front", "discard", "hop"):
            assert info[k] == 2 * ic[k], k
        assert info["fs_hz"] == 2 * BW * 1e6
        raw = torch.zeros(2 * 4096, dtype=torch.int8, device="cuda")
        prof = torch.zeros((4, 64), device="cuda")
        ser = torch.zeros(4096, device="cuda")
        # the complex entry points refuse a real plan and vice versa
        assert P.pond_dedisperse_fold(h, raw, 2048, 0, prof, 4) == P.POND_EINVAL
        assert P.pond_real_dedisperse(hc, raw, 2048, 0, prof, 4)[0] == P.POND_EINVAL
        with pytest.raises(P.PondError):
            P.pond_plan_expect(h, 2048, 0)
        # odd counts, misaligned input, bad decim
        assert P.pond_real_dedisperse(h, raw, 2047, 0, prof, 4)[0] == P.POND_EINVAL
        assert P.pond_real_dedisperse(h, raw, 2048, 1001, prof, 4)[0] == P.POND_EINVAL
        assert P.pond_real_dedisperse(h, raw.data_ptr() + 2, 2046, 0, prof, 4)[0] == P.POND_EINVAL
        for d in (1, 3, 64):
            assert P.pond_real_dedisperse(h, raw, 2048, 0, prof, 4, d, ser, 4096)[0] == P.POND_EINVAL
        # a short valid call produces nothing yet and advances the position
        assert P.pond_real_expect(h, 4096, 0) == (0, 0)
        assert P.pond_real_dedisperse(h, raw, 4096, 0, prof, 4, 32, ser, 4096) == (0, 0)
        torch.cuda.synchronize()
        assert P.pond_plan_query(h)["samples_in"] == 4096
    finally:
        P.pond_plan_destroy(h)
        P.pond_plan_destroy(hc)
    for prec in (P.POND_MIXED, P.POND_HALF):
        with pytest.raises(P.PondError):
            P.pond_real_plan_create(F0, BW, 3.1, 1 << 20, 64, 3.3e-2, prec, 0, "lsb")
    with pytest.raises(P.PondError):
        P.pond_real_plan_create(F0, BW, 3.1, (1 << 20) + 2, 64, 3.3e-2, P.POND_FP32, 0, "lsb")
    with pytest.raises(P.PondError):
        P.pond_real_plan_create(F0, BW, 3.1, 1 << 20, 64, 3.3e-2, P.POND_FP32, 0, 7)


def test_real_full_stream_sampled_blocks():
    """The 60 s real stream as the benchmark times it (1.92e9 real samples,
    real blocks of 2^24 at DM 50, one call): the series of the first,
    a middle and the last block against the oracle's real path run on just
    that block's input."""
    import torch
    import paper_1503_01405_amd as P
    nfft, dm, nsamp, decim = 1 << 24, 50.0, 1_920_000_000, 32
    print("case: real full stream 60 s", flush=True)
    raw = synth.pulsed_stream_int8(2, nsamp, fs_hz=2 * BW * 1e6, sigma=synth.SIGMA / 2 ** 0.5)
    x = torch.from_numpy(raw).to("cuda")
    res = {}
    for precision in ("mixed_valu", "fp32"):
        plan = P.Plan(F0, BW, dm, nfft, 1024, 0.0891, precision=precision, subint_nsamp=320_000_000,
                      decim=decim, sideband="lsb")
        hop_r = plan.info()["hop"]
        _, ser = plan.process(x)
        plan.flush(device=x.device)
        torch.cuda.synchronize()
        res[precision] = ser.cpu().numpy()
        plan.close()
    del x
    nb = (nsamp - nfft) // hop_r + 1
    for b in (0, nb // 2, nb - 1):
        r = O.run_real(raw[2 * b * hop_r:2 * (b * hop_r + nfft)], F0, BW, dm, nfft // 2, 1024, 0.0891,
                       sideband="lsb", decim=decim)
        want = r["series"]
        for precision, ser in res.items():
            got = ser[b * hop_r // decim:(b + 1) * hop_r // decim]
            e = rel_l2(got, want)
            print(f"block {b} {precision}: series rel-L2 {e:.3e}", flush=True)
            assert e <= TOL[precision][1], (b, precision, e)
