"""Serving loop: streams admitted against a device-memory budget, blocks
submitted as they arrive and run concurrently on the device.  Each stream's
profiles in the mix must equal, bit for bit, those of the same blocks run
alone on a plan of its own (the fold accumulates in integers, so neither
the interleaving nor the batching changes a result), and one stream is
checked against the oracle."""
import random
import time

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import BW, F0

# (dm, nfft, nbins, period_s, subint_nsamp, precision)
STREAMS = [
    (0.5, 1 << 16, 64, 2.1e-3, 300_000, "fp32"),
    (3.0, 1 << 19, 128, 0.033, 1_000_000, "mixed_valu"),
    (12.0, 1 << 21, 256, 0.25, 0, "mixed"),
    (1.2, 1 << 18, 100, 0.0891, 700_000, "half"),
    (25.0, 1 << 22, 512, 1.3, 2_000_000, "fp32"),
]
NSAMP = 6_000_000
MAX_BLOCK = 1_200_000


def _desc(P, s, max_block=MAX_BLOCK):
    dm, nfft, nbins, period, subint, prec = s
    return P.stream_desc(F0, BW, dm, nfft, nbins, period, subint, max_block, prec)


def test_stream_bytes_is_host_arithmetic():
    import paper_1503_01405_amd as P
    d = _desc(P, STREAMS[4])
    b = P.pond_server_stream_bytes(d)
    # at least the staging, the work area of one block and the table
    assert b >= 2 * MAX_BLOCK * 2 + (1 << 22) * 8 + (1 << 22) * 16
    bad = _desc(P, STREAMS[4])
    bad.nfft = 3000
    assert P.pond_server_stream_bytes(bad) == P.POND_EINVAL
    bad = _desc(P, STREAMS[4], max_block=0)
    assert P.pond_server_stream_bytes(bad) == P.POND_EINVAL


def _blocks(seed, nsamp):
    rng = random.Random(seed)
    sizes, left = [], nsamp
    while left > 0:
        n = min(left, rng.randrange(150_000, MAX_BLOCK + 1, 2))
        sizes.append(n)
        left -= n
    return sizes


def _pinned(iq):
    import torch
    t = torch.empty(iq.size, dtype=torch.int8, pin_memory=True)
    t.numpy()[:] = iq
    return t


def _alone(P, s, iq, sizes):
    """The same blocks through pond_dedisperse_fold on one plan, then flush."""
    import torch
    dm, nfft, nbins, period, subint, prec = s
    plan = P.Plan(F0, BW, dm, nfft, nbins, period, precision=prec, subint_nsamp=subint)
    x = torch.from_numpy(iq).to("cuda")
    out, pos = [], 0
    for n in sizes:
        prof, _ = plan.process(x[2 * pos:2 * (pos + n)], want_series=False)
        out.append(prof.cpu().numpy())
        pos += n
    out.append(plan.flush(device=x.device).cpu().numpy())
    torch.cuda.synchronize()
    plan.close()
    return np.concatenate(out)


def _serve(P, streams, data, sizes, order, pace):
    import torch
    torch.cuda.init()   # torch's device state first, then the library's
    srv = P.pond_server_create(64 << 30, 16)
    try:
        ids = [P.pond_server_open(srv, _desc(P, s)) for s in streams]
        assert all(i >= 0 for i in ids), ids
        pinned = [_pinned(iq) for iq in data]
        pos = [0] * len(streams)
        k = [0] * len(streams)
        done = []
        rng = random.Random(5)
        for si in order:
            n = sizes[si][k[si]]
            t = P.pond_server_submit(srv, ids[si], pinned[si][2 * pos[si]:], n)
            assert t >= 0, t
            pos[si] += n
            k[si] += 1
            done += P.pond_server_poll(srv)
            if pace:
                time.sleep(rng.random() * 2e-3)
        q = P.pond_server_query(srv)
        assert q["open_streams"] == len(streams)
        while True:
            got = P.pond_server_poll(srv, wait=True)
            if not got:
                break
            done += got
        for i in ids:
            assert P.pond_server_close(srv, i) == P.POND_OK
        done += P.pond_server_poll(srv)
        profs = [P.pond_server_take_profiles(srv, i, s[2]) for i, s in zip(ids, streams)]
        assert P.pond_server_query(srv)["used_bytes"] == 0
        return profs, done
    finally:
        P.pond_server_destroy(srv)


@pytest.mark.gpu
@pytest.mark.parametrize("pace", [True, False], ids=["paced", "burst"])
def test_mix_equals_alone(pace):
    import paper_1503_01405_amd as P
    print(f"case: serve mix vs alone pace={pace} streams={len(STREAMS)}", flush=True)
    data = [synth.white_stream_int8(40 + i, NSAMP) for i in range(len(STREAMS))]
    sizes = [_blocks(100 + i, NSAMP) for i in range(len(STREAMS))]
    order = [i for i in range(len(STREAMS)) for _ in sizes[i]]
    random.Random(7).shuffle(order)
    profs, done = _serve(P, STREAMS, data, sizes, order, pace)
    assert len(done) == sum(len(s) for s in sizes)
    assert all(c["status"] == P.POND_OK and c["latency_us"] > 0 for c in done)
    assert sum(c["n_profiles"] for c in done) + len(STREAMS) >= sum(p.shape[0] for p in profs)
    for i, s in enumerate(STREAMS):
        want = _alone(P, s, data[i], sizes[i])
        assert profs[i].shape == want.shape, (i, profs[i].shape, want.shape)
        np.testing.assert_array_equal(profs[i], want, err_msg=f"stream {i}")


@pytest.mark.gpu
def test_served_stream_matches_oracle():
    import paper_1503_01405_amd as P
    s = STREAMS[0]
    print("case: served stream vs oracle", flush=True)
    iq = synth.white_stream_int8(40, NSAMP)
    sizes = _blocks(100, NSAMP)
    profs, _ = _serve(P, [s], [iq], [sizes], [0] * len(sizes), False)
    dm, nfft, nbins, period, subint, _ = s
    ref = O.run(iq, F0, BW, dm, nfft, nbins, period, subint_nsamp=subint, decim=16, workers=8)
    want = ref["profiles"][:ref["complete"] + 1]
    got = profs[0]
    assert got.shape == want.shape
    err = max(np.linalg.norm(got[j] - want[j]) / np.linalg.norm(want[j]) for j in range(got.shape[0]))
    assert err <= 1e-6, err


@pytest.mark.gpu
def test_admission_by_budget():
    import paper_1503_01405_amd as P
    print("case: serve admission", flush=True)
    import torch
    torch.cuda.init()
    d = _desc(P, STREAMS[4])
    need = P.pond_server_stream_bytes(d)
    srv = P.pond_server_create(need + need // 2, 8)
    try:
        a = P.pond_server_open(srv, d)
        assert a >= 0 and P.pond_server_stream_state(srv, a) == P.POND_STREAM_OPEN
        q = P.pond_server_query(srv)
        assert 0 < q["used_bytes"] <= need
        # a second such stream is admitted with fewer blocks per launch, or waits
        b = P.pond_server_open(srv, d)
        assert b >= 0
        if P.pond_server_stream_state(srv, b) == P.POND_STREAM_OPEN:
            assert P.pond_server_query(srv)["used_bytes"] <= need + need // 2
        assert P.pond_server_close(srv, b) == P.POND_OK
        c = P.pond_server_open(srv, _desc(P, STREAMS[4], max_block=need))  # staging alone exceeds it
        assert c == P.POND_EBUSY
        assert P.pond_server_close(srv, a) == P.POND_OK
        assert P.pond_server_query(srv)["used_bytes"] == 0
        a2 = P.pond_server_open(srv, d)
        assert a2 >= 0
        assert P.pond_server_close(srv, a2) == P.POND_OK
    finally:
        P.pond_server_destroy(srv)


@pytest.mark.gpu
def test_deferred_admission_runs_after_budget_frees():
    """Continuous batching under a budget: stream B does not fit while A is
    open, so it waits with the blocks submitted to it; closing A returns A's
    memory, B is admitted (reported by poll as an admission), its queued
    blocks run, and both streams' profiles equal the same blocks run alone.
    A third stream closed before its admission has its blocks cancelled."""
    import paper_1503_01405_amd as P
    import torch
    print("case: serve deferred admission", flush=True)
    torch.cuda.init()
    sa, sb = STREAMS[4], STREAMS[2]
    da, db = _desc(P, sa), _desc(P, sb)
    need_a, need_b = P.pond_server_stream_bytes(da), P.pond_server_stream_bytes(db)
    srv = P.pond_server_create(need_a + need_b // 4, 8)
    try:
        a = P.pond_server_open(srv, da)
        b = P.pond_server_open(srv, db)
        c = P.pond_server_open(srv, db)
        assert P.pond_server_stream_state(srv, a) == P.POND_STREAM_OPEN
        assert P.pond_server_stream_state(srv, b) == P.POND_STREAM_WAITING
        assert P.pond_server_stream_state(srv, c) == P.POND_STREAM_WAITING
        data = {a: synth.white_stream_int8(60, NSAMP), b: synth.white_stream_int8(61, NSAMP)}
        sizes = {a: _blocks(160, NSAMP), b: _blocks(161, NSAMP)}
        pinned = {k: _pinned(v) for k, v in data.items()}
        tickets = {a: [], b: []}
        for k in (a, b):
            pos = 0
            for n in sizes[k]:
                t = P.pond_server_submit(srv, k, pinned[k][2 * pos:], n)
                assert t >= 0, t
                tickets[k].append(t)
                pos += n
        cz = P.pond_server_submit(srv, c, pinned[b], 1000)
        assert cz >= 0
        done = []
        while True:
            got = P.pond_server_poll(srv, wait=True)
            if not got:
                break
            done += got
        # all of A's blocks ran; none of B's, which still waits
        assert sorted(x["ticket"] for x in done if x["stream"] == a) == tickets[a]
        assert not [x for x in done if x["stream"] == b]
        assert P.pond_server_stream_state(srv, b) == P.POND_STREAM_WAITING
        assert P.pond_server_close(srv, c) == P.POND_OK      # never admitted: cancelled
        assert P.pond_server_stream_state(srv, c) == P.POND_STREAM_CLOSED
        assert P.pond_server_stream_state(srv, b) == P.POND_STREAM_WAITING
        assert P.pond_server_close(srv, a) == P.POND_OK      # frees A's memory: B is admitted
        assert P.pond_server_stream_state(srv, b) == P.POND_STREAM_OPEN
        while True:
            got = P.pond_server_poll(srv, wait=True)
            if not got:
                break
            done += got
        adm = [x for x in done if x["ticket"] == P.POND_TICKET_ADMITTED]
        assert [(x["stream"], x["status"]) for x in adm] == [(b, P.POND_OK)]
        assert sorted(x["ticket"] for x in done if x["stream"] == b and x["ticket"] >= 0) == tickets[b]
        assert all(x["status"] == P.POND_OK for x in done if x["stream"] in (a, b))
        assert [(x["ticket"], x["status"]) for x in done if x["stream"] == c] == [(cz, P.POND_ECANCELED)]
        assert P.pond_server_close(srv, b) == P.POND_OK
        profs = {k: P.pond_server_take_profiles(srv, k, s[2]) for k, s in ((a, sa), (b, sb))}
        assert P.pond_server_query(srv)["used_bytes"] == 0
    finally:
        P.pond_server_destroy(srv)
    for k, s in ((a, sa), (b, sb)):
        want = _alone(P, s, data[k], sizes[k])
        assert profs[k].shape == want.shape
        np.testing.assert_array_equal(profs[k], want, err_msg=f"stream {k}")
