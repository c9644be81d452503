"""Blocks-per-launch autotuner (pond_plan_create_ex with POND_BATCH_AUTOTUNE)
and its POND_AUTOTUNE_CACHE file."""
import os

import numpy as np
import pytest

import synth
from gpu_helpers import BW, F0, gpu_run


def test_autotune_query_rejects_null_plan():
    import paper_1503_01405_amd as P
    with pytest.raises(P.PondError):
        P.pond_plan_autotune(None)


@pytest.mark.gpu
def test_autotune_measures_caches_and_matches_default(tmp_path, monkeypatch):
    import paper_1503_01405_amd as P
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("POND_AUTOTUNE_CACHE", str(cache))
    nfft, dm = 1 << 20, 10.0
    print("case: autotune nfft=2^20 half, measure", flush=True)
    a = P.Plan(F0, BW, dm, nfft, 512, synth.PERIOD_S, precision="half", max_batch=P.POND_BATCH_AUTOTUNE)
    r = a.autotune()
    a.close()
    print(r, flush=True)
    assert r["batch"] in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32) and not r["from_cache"]
    assert r["ms_per_block"] > 0 and r["default_ms_per_block"] > 0
    assert r["default_batch"] == 16  # 2^29 bytes of float16 pairs, capped at 16
    # the choice is no slower than the default by more than the 2% margin
    assert r["ms_per_block"] <= r["default_ms_per_block"] * 1.02 + 1e-9
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and f"nfft={nfft}" in lines[0] and f"batch={r['batch']} " in lines[0]
    print("case: autotune from cache", flush=True)
    b = P.Plan(F0, BW, dm, nfft, 512, synth.PERIOD_S, precision="half", max_batch=P.POND_BATCH_AUTOTUNE)
    rb = b.autotune()
    b.close()
    assert rb["from_cache"] and rb["batch"] == r["batch"]
    assert len(cache.read_text().splitlines()) == 1
    # a plan made without the tuner has no result
    c = P.Plan(F0, BW, dm, nfft, 512, synth.PERIOD_S, precision="half")
    with pytest.raises(P.PondError):
        c.autotune()
    c.close()
    # the tuned plan computes the same bits as the default one (the fold is
    # exact integer arithmetic, so the launch size cannot change a result)
    nsamp = 5 * nfft
    iq = synth.white_stream_int8(5, nsamp)
    print("case: autotuned vs default output", flush=True)
    t = gpu_run(iq, dm, nfft, 512, synth.PERIOD_S, precision="half", max_batch=P.POND_BATCH_AUTOTUNE)
    d = gpu_run(iq, dm, nfft, 512, synth.PERIOD_S, precision="half")
    assert np.array_equal(t[0], d[0]) and np.array_equal(t[1], d[1])


@pytest.mark.gpu
def test_autotune_with_unwritable_cache_still_tunes(tmp_path, monkeypatch):
    import paper_1503_01405_amd as P
    monkeypatch.setenv("POND_AUTOTUNE_CACHE", str(tmp_path / "missing_dir" / "tune.txt"))
    print("case: autotune unwritable cache", flush=True)
    p = P.Plan(F0, BW, 1.0, 1 << 18, 256, synth.PERIOD_S, precision="fp32", max_batch=P.POND_BATCH_AUTOTUNE)
    r = p.autotune()
    p.close()
    assert r["batch"] >= 1 and not r["from_cache"]
    assert not os.path.exists(tmp_path / "missing_dir")


@pytest.mark.gpu
def test_search_autotune_per_group_and_same_profiles(monkeypatch):
    """A search created with POND_BATCH_AUTOTUNE tunes each length group
    and folds the same bits as the default search (integer fold)."""
    import torch
    import paper_1503_01405_amd as P
    monkeypatch.delenv("POND_AUTOTUNE_CACHE", raising=False)
    dms = [0.0, 0.5, 1.0, 2.0]
    nsamp = 3_000_000
    iq = synth.white_stream_int8(11, nsamp)
    x = torch.from_numpy(iq).to("cuda")
    outs = []
    for mb in (None, P.POND_BATCH_AUTOTUNE):
        print(f"case: search autotune={mb}", flush=True)
        h = P.pond_search_create(F0, BW, dms, 128, synth.PERIOD_S, 1 << 16, 1 << 19, P.POND_HALF, max_batch=mb)
        try:
            groups = sorted({P.pond_search_trial(h, t)[0] for t in range(len(dms))})
            if mb is None:
                with pytest.raises(P.PondError):
                    P.pond_search_autotune(h, groups[0])
            else:
                for n in groups:
                    r = P.pond_search_autotune(h, n)
                    print(n, r, flush=True)
                    assert r["batch"] >= 1 and r["ms_per_block"] > 0 and r["default_ms_per_block"] > 0
                with pytest.raises(P.PondError):
                    P.pond_search_autotune(h, 1 << 12)  # no such group
            out = torch.empty((len(dms), 128), dtype=torch.float32, device="cuda")
            assert P.pond_search_run(h, x, nsamp, out) == P.POND_OK
            torch.cuda.synchronize()
            outs.append(out.cpu().numpy())
        finally:
            P.pond_search_destroy(h)
    assert np.array_equal(outs[0], outs[1])
