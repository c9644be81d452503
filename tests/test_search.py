"""DM-trial search: grouping rule, oracle behaviour on a dispersed pulse
(CPU), GPU parity with the oracle per trial, and the S/N-vs-DM peak of the
batched search on the GPU."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import BW, EPS_HALF, F0, dispersed_pulsar_stream, profile_rel_l2

TRIALS_128 = np.arange(128) * 0.5


def test_search_groups_of_the_128_trial_workload():
    """N_t = clamp(2 discard_t, 2^20, 2^23): four length groups, DM 0-8.5,
    9-17, 17.5-34 and 34.5-63.5, each with hop = N/2."""
    geo = O.search_geometry(F0, BW, TRIALS_128)
    by_n = {}
    for t in geo:
        by_n.setdefault(t["nfft"], []).append(t["dm"])
        assert t["hop"] == t["nfft"] // 2
        g = O.plan_geometry(F0, BW, t["dm"], t["nfft"])
        assert g["discard"] <= t["hop"] and t["n_front"] == g["n_front"]
    assert sorted(by_n) == [1 << 20, 1 << 21, 1 << 22, 1 << 23]
    assert (min(by_n[1 << 20]), max(by_n[1 << 20])) == (0.0, 8.5)
    assert (min(by_n[1 << 21]), max(by_n[1 << 21])) == (9.0, 17.0)
    assert (min(by_n[1 << 22]), max(by_n[1 << 22])) == (17.5, 34.0)
    assert (min(by_n[1 << 23]), max(by_n[1 << 23])) == (34.5, 63.5)


def test_oracle_search_snr_peaks_at_true_dm():
    """A pulse dispersed at DM 2.0 is sharpest when folded at DM 2.0."""
    iq = dispersed_pulsar_stream(4, 2_000_000, 2.0, period=0.02)
    dms = np.arange(1.5, 2.51, 0.25)
    profs, geo = O.search(iq, F0, BW, dms, 256, 0.02, nfft_min=1 << 16, nfft_max=1 << 20,
                          workers=8)
    snr = [O.profile_snr(p) for p in profs]
    assert dms[int(np.argmax(snr))] == 2.0, snr


def _gpu_search(iq, dms, nbins, period, nmin, nmax, precision):
    import torch
    import paper_1503_01405_amd as P
    x = torch.from_numpy(iq).to("cuda")
    prec = P.FORMS[precision]
    h = P.pond_search_create(F0, BW, dms, nbins, period, nmin, nmax, prec)
    try:
        out = torch.zeros((len(dms), nbins), device="cuda")
        assert P.pond_search_run(h, x, iq.size // 2, out) == P.POND_OK
        torch.cuda.synchronize()
        geo = [P.pond_search_trial(h, t) for t in range(len(dms))]
        return out.cpu().numpy(), geo
    finally:
        P.pond_search_destroy(h)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_valu", "half"])
def test_gpu_search_parity(precision):
    dms = [0.0, 0.4, 1.1, 2.5, 3.0, 6.0]
    nbins, period, nmin, nmax = 128, 3.3e-3, 1 << 14, 1 << 20
    print(f"case: search parity {precision} dms={dms}", flush=True)
    iq = synth.white_stream_int8(31, 1_500_001)
    want, geo = O.search(iq, F0, BW, dms, nbins, period, nfft_min=nmin, nfft_max=nmax, workers=8)
    got, ggeo = _gpu_search(iq, dms, nbins, period, nmin, nmax, precision)
    assert [(t["nfft"], t["n_front"], t["hop"]) for t in geo] == ggeo
    err = profile_rel_l2(got, want)
    tol = 1e-6 if precision == "fp32" else 1e-4
    if precision in ("half", "mixed"):
        # plus float16 rounding noise over the samples of a bin (as in the
        # single-DM parity tests): 3 * 5e-3 / sqrt(samples per bin)
        nsamp = iq.size // 2
        n_out = min(((nsamp - t["nfft"]) // t["hop"] + 1) * t["hop"] for t in geo)
        tol += 3 * 5e-3 / np.sqrt(n_out / nbins)
    print(f"{precision}: max per-trial profile rel-L2 {err:.3e} (tol {tol:.1e})")
    assert err <= tol


@pytest.fixture(scope="module")
def production_groups_case():
    """Trials in the three longest length groups of the 128-trial workload
    (2^21 for DM 9-17, 2^22 for 17.5-34, 2^23 for 34.5-63.5), two per
    group, over three 2^23 blocks of a pulsed stream; oracle per trial."""
    dms = [9.0, 13.5, 20.0, 33.5, 37.0, 63.5]
    nbins, period, nmin, nmax = 512, synth.PERIOD_S, 1 << 20, 1 << 23
    nsamp = (1 << 23) + 2 * (1 << 22) + 4321
    iq = synth.pulsed_stream_int8(17, nsamp)
    want, geo = O.search(iq, F0, BW, dms, nbins, period, nfft_min=nmin, nfft_max=nmax, workers=16)
    assert sorted({t["nfft"] for t in geo}) == [1 << 21, 1 << 22, 1 << 23]
    return iq, dms, nbins, period, nmin, nmax, want, geo


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "mixed", "mixed_valu", "half"])
def test_gpu_search_parity_production_groups(production_groups_case, precision):
    """Row passes of 2^11-2^13 (kRowFwd / kRowInv, the float16 per-stage LDS
    layouts of rows >= 2^12) against the oracle, trial by trial."""
    iq, dms, nbins, period, nmin, nmax, want, geo = production_groups_case
    print(f"case: search parity, production groups, {precision}", flush=True)
    got, ggeo = _gpu_search(iq, dms, nbins, period, nmin, nmax, precision)
    assert [(t["nfft"], t["n_front"], t["hop"]) for t in geo] == ggeo
    nsamp = iq.size // 2
    for t, (g, tr) in enumerate(zip(got, geo)):
        n_out = ((nsamp - tr["nfft"]) // tr["hop"] + 1) * tr["hop"]
        tol = 1e-6 if precision == "fp32" else 1e-4
        if precision in ("half", "mixed"):
            tol += 3 * EPS_HALF / np.sqrt(n_out / nbins)
        e = profile_rel_l2(g[None], want[t][None])
        gain = float(g.sum() / want[t].sum())   # bins hold nearly equal counts
        print(f"{precision}: DM {dms[t]} N=2^{tr['nfft'].bit_length() - 1} rel-L2 {e:.3e} (tol {tol:.1e}) "
              f"gain {gain - 1:+.2e}", flush=True)
        assert e <= tol, (dms[t], e)
        assert abs(gain - 1) <= 2e-5 + 3 * EPS_HALF / np.sqrt(n_out), (dms[t], gain)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "half"])
def test_gpu_search_graph_replay_matches_eager(precision):
    """pond_search_run captured once into a HIP graph and replayed: every
    replay equals the eager profiles bitwise (integer fold), with eager
    searches and synchronisation in between."""
    import torch
    import paper_1503_01405_amd as P
    dms = [0.0, 1.5, 4.0, 9.5]
    nbins, period, nmin, nmax = 256, 7.7e-3, 1 << 16, 1 << 21
    nsamp = 3_000_017
    print(f"case: search graph replay {precision}", flush=True)
    x = torch.from_numpy(synth.white_stream_int8(41, nsamp)).to("cuda")
    h = P.pond_search_create(F0, BW, dms, nbins, period, nmin, nmax, P.FORMS[precision])
    try:
        out = torch.zeros((len(dms), nbins), device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            assert P.pond_search_run(h, x, nsamp, out, s) == P.POND_OK
        torch.cuda.synchronize()
        ref = out.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            assert P.pond_search_run(h, x, nsamp, out, torch.cuda.current_stream()) == P.POND_OK
        for rep in range(3):
            out.fill_(-1.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy(), err_msg=f"replay {rep}")
            with torch.cuda.stream(s):
                assert P.pond_search_run(h, x, nsamp, out, s) == P.POND_OK
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
        del g
    finally:
        P.pond_search_destroy(h)


@pytest.mark.gpu
def test_gpu_search_finds_dm_37_2():
    """The batched-search workload's structure: a pulse dispersed at DM 37.2,
    trials every 0.5 with FFT lengths by smear (2^23 here); the S/N peaks at
    37.0, the trial nearest 37.2 (residual DM 0.2 against 0.3 at 37.5)."""
    print("case: search S/N peak DM 37.2", flush=True)
    iq = dispersed_pulsar_stream(9, 64_000_000, 37.2)
    dms = list(np.arange(35.0, 39.51, 0.5))
    got, _ = _gpu_search(iq, dms, 512, synth.PERIOD_S, 1 << 20, 1 << 23, "half")
    snr = [O.profile_snr(p) for p in got]
    print("S/N:", [f"{d}:{s:.1f}" for d, s in zip(dms, snr)])
    assert dms[int(np.argmax(snr))] == 37.0
    assert max(snr) > 1.5 * snr[0]
