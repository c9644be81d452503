"""Throughput of the coherent-dedispersion + fold path on one MI355X.

Workload (the production configuration): a continuous 60 s stream of
single-polarisation complex int8 baseband at 16 Msps centred on 326.5 MHz
(960,000,000 samples, 1.92 GB resident in HBM), dedispersed at DM 50 with
overlap-save FFTs of 2^23 points (2^22 discarded per block: 227 blocks,
952,107,008 valid outputs), detected, decimated to 1 us and folded at
P = 0.0891 s into 1024 bins per 10 s sub-integration.

One step = the whole stream through the C ABI (pond_dedisperse_series on
all 960M samples, then the end-of-stream flush) = every kernel of the path.
Both precision forms are timed; `value` is the mixed form's Msamples/s of
valid outputs, with the float32 form and the speed-up beside it.

Prints ONE JSON line.

`--workload serve` runs the serving loop: 16 concurrent streams (DM
log-uniform 0.5-200, period uniform 2 ms-2 s, FFT length by smear between
2^16 and 2^24) fed 1 s int8 blocks from pinned host memory.  A paced run
(blocks arriving once a second per stream with exponential jitter) gives
p50/p99 block latency; a saturated run (every block queued at once) gives
the aggregate throughput and real-time factor.

`--workload aid` times the incoherent (filterbank) mode on the same 60 s
stream: 1024 channels, 4 spectra per integrated sample (256 us), channel
delays of Eq. (3) at DM 50, 1024 bins.

`--workload real` times the real two-channel input path (channels A and B
added in phase, packed real-to-complex transforms): 60 s of int8 A/B pairs
at 32 Msps real (1,920,000,000 real samples, 3.84 GB resident), DM 50,
real blocks of 2^24 (packed 2^23), 1 us series, 1024 bins per 10 s.

`--workload search` times the batched DM-trial search instead: a 10 s
stream of the same generator (160,000,000 samples) folded at 128 trial DMs
0-63.5 in steps of 0.5 into 512 bins, FFT length per trial by smear
(2^20-2^23, four length groups, one shared forward transform per group and
block).  Its line reports trial-samples/s (trials x stream samples per
second of the whole search) and the stream's real-time factor.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

F0, BW, DM, NFFT, NBINS, PERIOD = 326.5, 16.0, 50.0, 1 << 23, 1024, 0.0891
NSAMP = 960_000_000
SUBINT = 160_000_000   # 10 s of outputs
DECIM = 16             # 1 us
SEED = 2
METRIC = "Msamples/s dedispersed+folded at DM 50 (×realtime), mixed-prec vs FP32 form"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, blocks, elem, nfft, hop):
    """Bytes each kernel must move per the three-pass design, for `blocks`
    overlap-save blocks: int8 input (2 B/sample) read once per block,
    complex intermediates of `elem` bytes written/read once per pass,
    1 us series (4 B per 16 outputs) written once."""
    if kernel == "k1_unpack_colfft":
        return blocks * nfft * (2 + elem)
    if kernel == "k2_row":
        return blocks * nfft * 2 * elem
    if kernel == "k3_colinv_detect_fold":
        return blocks * (nfft * elem + hop // 16 * 4)
    return 0


def copy_bandwidth(nbytes=1 << 31, reps=10):
    """Achievable HBM bandwidth (GB/s, bytes read + written) of the
    library's own streaming copy kernel over nbytes, event-timed."""
    import torch
    import paper_1503_01405_amd as P
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    P.pond_copy_device(dst, src, nbytes, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        P.pond_copy_device(dst, src, nbytes, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / 1e3) / 1e9


def kernel_source_hash():
    """sha256[:16] over the device code of the library: the .hip sources and
    the headers they include, transitively (as recorded in the committed
    rocprofv3 summaries; host-only changes leave it as it is)."""
    import hashlib
    import re
    d = os.path.join(ROOT, "paper_1503_01405_amd", "csrc")
    files = {f for f in os.listdir(d) if f.endswith(".hip")}
    todo = sorted(files)
    while todo:
        with open(os.path.join(d, todo.pop()), encoding="utf-8") as fh:
            for inc in re.findall(r'^#include "([^"]+)"', fh.read(), re.M):
                if inc not in files and os.path.exists(os.path.join(d, inc)):
                    files.add(inc)
                    todo.append(inc)
    h = hashlib.sha256()
    for f in sorted(files):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_prefix, form, max_batch):
    """HBM bytes per overlap-save block of a kernel (read, written) from the
    committed counter summary of that form at the run's blocks per launch,
    or None if there is none or it was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_bytes_dm50_nfft2e23_{form}_b{max_batch}.txt")
    if not os.path.exists(path):
        return None
    src = None
    with open(path) as fh:
        lines = fh.read().splitlines()
    for ln in lines:
        if ln.startswith("kernel source sha256[:16]:"):
            src = ln.split("]:", 1)[1].split()[0]
    if src != kernel_source_hash():
        return None
    for ln in lines:
        if ln.startswith("TRAFFIC ") and kernel_prefix in ln:
            kv = dict(t.split("=") for t in ln.split() if "=" in t)
            return float(kv["fetch_bytes_per_block"]), float(kv["write_bytes_per_block"])
    return None


def run_form(precision, x, steps, warmup, graph=False, max_batch=0):
    import torch
    import paper_1503_01405_amd as P

    # blocks per launch chosen by the library's autotuner at plan creation
    # (outside the timed region; POND_AUTOTUNE_CACHE, if set, holds it),
    # unless given (--max-batch, for counter runs with a fixed launch shape)
    plan = P.Plan(F0, BW, DM, NFFT, NBINS, PERIOD, precision=precision, subint_nsamp=SUBINT, decim=DECIM,
                  max_batch=max_batch if max_batch > 0 else P.POND_BATCH_AUTOTUNE)
    info = plan.info()
    tune = plan.autotune() if max_batch <= 0 else None
    nsamp = x.numel() // 2
    nprof, nout = P.pond_plan_expect(plan.handle, nsamp, SUBINT)
    prof = torch.empty((nprof + 1, NBINS), dtype=torch.float32, device=x.device)
    ser = torch.empty(nout // DECIM, dtype=torch.float32, device=x.device)
    stream = torch.cuda.current_stream()

    def step():
        r, ns = P.pond_dedisperse_series(plan.handle, x, nsamp, SUBINT, prof, nprof, DECIM, ser,
                                         ser.numel(), stream)
        if r != nprof or ns != ser.numel():
            raise RuntimeError(f"unexpected call result {r} {ns}")
        r = P.pond_dedisperse_fold(plan.handle, None, 0, SUBINT, prof[nprof:], 1, stream)
        if r != 1:
            raise RuntimeError(f"flush returned {r}")

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    ev_ms = ev0.elapsed_time(ev1) / steps
    ms = max(wall, ev_ms)
    # per-kernel times from a second pass with every launch bracketed by
    # events on the plan's stream (kept out of the timed steps above, since
    # the event records themselves cost time between launches)
    P.pond_plan_set_timing(plan.handle, True)
    for _ in range(steps):
        step()
    kt = P.pond_plan_kernel_times(plan.handle)
    P.pond_plan_set_timing(plan.handle, False)
    res = dict(ms_per_step=ms, ms_events=ev_ms, ms_wall=wall, outputs=nout, kernels=kt, info=info, tune=tune)
    if graph:
        # the same step captured once into a HIP graph and replayed
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            stream = torch.cuda.current_stream()
            step()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        del g
    plan.close()
    return res


def host_cpu():
    """The host the CPU baseline ran on: logical CPUs and the processor model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(host_cpus=os.cpu_count(), cpu_model=model)


def cpu_baseline(iq_np, nblocks):
    """The FP64 oracle, as it stands, on the first `nblocks` blocks."""
    import oracle as O
    workers = max(1, min(16, os.cpu_count() or 1))
    g = O.plan_geometry(F0, BW, DM, NFFT)
    n_in = NFFT + (nblocks - 1) * g["hop"]
    sub = iq_np[:2 * n_in]
    t0 = time.perf_counter()
    r = O.run(sub, F0, BW, DM, NFFT, NBINS, PERIOD, subint_nsamp=SUBINT, decim=DECIM, workers=workers)
    dt = time.perf_counter() - t0
    msps = r["n_out"] / dt / 1e6
    return dict(value=round(msps, 3), unit="Msamples/s", cores=workers, kind="oracle", **host_cpu(),
                sample=f"first {nblocks} of 227 overlap-save blocks ({r['n_out']} outputs, "
                       f"{r['n_out'] / 16e6:.2f} s of data) of the same stream, {dt:.1f} s of CPU work",
                xrealtime=round(msps / 16.0, 3))


SEARCH_NSAMP = 160_000_000
SEARCH_NBINS = 512
SEARCH_METRIC = "DM-trial Msamples/s (128 trials, DM 0-63.5, 10 s stream, 512 bins)"


def search_bytes(geo_groups, nsamp, elem):
    """Bytes the search's passes must move for one stream: per group and
    block, K1 (int8 read + spectrum write) and the forward row pass (read +
    write), then per trial the inverse row pass (read + write) and K3
    (read)."""
    total = 0
    for nfft, hop, ntr in geo_groups:
        nb = 0 if nsamp < nfft else (nsamp - nfft) // hop + 1
        total += nb * nfft * ((2 + elem) + 2 * elem + ntr * (3 * elem))
    return total


def run_search(precision, x, dms, steps, warmup):
    import torch
    import paper_1503_01405_amd as P
    prec = P.FORMS[precision]
    h = P.pond_search_create(F0, BW, dms, SEARCH_NBINS, PERIOD, 1 << 20, 1 << 23, prec,
                             max_batch=P.POND_BATCH_AUTOTUNE)
    nsamp = x.numel() // 2
    out = torch.empty((len(dms), SEARCH_NBINS), dtype=torch.float32, device=x.device)
    stream = torch.cuda.current_stream()
    try:
        geo = [P.pond_search_trial(h, t) for t in range(len(dms))]
        tune = {n: P.pond_search_autotune(h, n) for n in sorted({g[0] for g in geo})}
        for _ in range(warmup):
            if P.pond_search_run(h, x, nsamp, out, stream) != P.POND_OK:
                raise RuntimeError("pond_search_run failed")
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            if P.pond_search_run(h, x, nsamp, out, stream) != P.POND_OK:
                raise RuntimeError("pond_search_run failed")
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps * 1e3
        ms = max(wall, ev0.elapsed_time(ev1) / steps)
    finally:
        P.pond_search_destroy(h)
    groups = {}
    for n, _, hop in geo:
        groups.setdefault((n, hop), 0)
        groups[(n, hop)] += 1
    return dict(ms_per_step=ms, groups=[(n, hop, c) for (n, hop), c in sorted(groups.items())], tune=tune)


def search_cpu_baseline(iq_np, dms):
    """The FP64 oracle's search, as it stands, on one trial of each FFT-length
    group over the first 2^24 + 2^22 samples of the stream."""
    import oracle as O
    workers = max(1, min(16, os.cpu_count() or 1))
    geo = O.search_geometry(F0, BW, dms)
    pick, seen = [], set()
    for t in geo:
        if t["nfft"] not in seen:
            seen.add(t["nfft"])
            pick.append(t["dm"])
    n_in = (1 << 24) + (1 << 22)
    sub = iq_np[:2 * n_in]
    t0 = time.perf_counter()
    O.search(sub, F0, BW, pick, SEARCH_NBINS, PERIOD, workers=workers)
    dt = time.perf_counter() - t0
    v = len(pick) * n_in / dt / 1e6
    return dict(value=round(v, 3), unit="Msamples/s", cores=workers, kind="oracle", **host_cpu(),
                sample=f"{len(pick)} trials (DM {', '.join(str(d) for d in pick)}: one per FFT length) over the "
                       f"first {n_in} samples, {dt:.1f} s of CPU work")


def main_search(args):
    import numpy as np
    import torch
    import synth

    t = time.perf_counter()
    iq = synth.pulsed_stream_int8(SEED, SEARCH_NSAMP)
    log(f"generated {SEARCH_NSAMP} samples in {time.perf_counter() - t:.1f} s")
    x = torch.from_numpy(iq).to("cuda:0")
    dms = [0.5 * i for i in range(128)]
    # the search takes the four single-DM forms (bfloat16 storage is a
    # plan-only reported variant)
    forms = [f for f in args.forms.split(",") if f and f != "bf16"]
    res = {}
    for f in forms:
        res[f] = run_search(f, x, dms, args.steps, args.warmup)
        log(f"search {f}: {res[f]['ms_per_step']:.3f} ms/step groups {res[f]['groups']}")
    head = min(res, key=lambda f: res[f]["ms_per_step"]) if "fp32" not in res or len(res) == 1 else \
        min((f for f in res if f != "fp32"), key=lambda f: res[f]["ms_per_step"])
    h = res[head]
    value = len(dms) * SEARCH_NSAMP / (h["ms_per_step"] / 1e3) / 1e6
    elem = 8 if head == "fp32" else 4
    algo = search_bytes(h["groups"], SEARCH_NSAMP, elem)
    achieved = algo / (h["ms_per_step"] / 1e3) / 1e9
    out = {
        "metric": SEARCH_METRIC, "value": round(value, 1), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(h["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"mixed": "f16 (matrix-core DFT) / f32 accumulate", "mixed_valu": "f16-storage/f32",
                  "half": "f16 (packed VALU) / f32 detect+fold",
                  "fp32": "f32"}[head],
        "data": "synthetic",
        "config": {"workload": "10 s 16 Msps int8 I/Q at 326.5 MHz, 128 DM trials 0-63.5 step 0.5, "
                               "nfft 2^20-2^23 by smear, 512 bins", "nsamp": SEARCH_NSAMP, "ntrials": len(dms),
                   "groups_nfft_hop_trials": h["groups"], "form": head},
        "stream_xrealtime": round(SEARCH_NSAMP / 16e6 / (h["ms_per_step"] / 1e3), 2),
        "forms": {f: dict(ms_per_step=round(r["ms_per_step"], 3),
                          value=round(len(dms) * SEARCH_NSAMP / (r["ms_per_step"] / 1e3) / 1e6, 1),
                          autotune={str(n): dict(batch=t["batch"], ms_per_block=round(t["ms_per_block"], 4),
                                                 default_batch=t["default_batch"],
                                                 default_ms_per_block=round(t["default_ms_per_block"], 4))
                                    for n, t in r["tune"].items()})
                  for f, r in res.items()},
        "roofline": dict(bound="hbm", kernel="whole search step", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                         unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                         algorithmic_bytes_per_step=algo),
    }
    if not args.no_cpu_baseline:
        del x
        torch.cuda.empty_cache()
        out["cpu_baseline"] = search_cpu_baseline(iq, dms)
    print(json.dumps(out), flush=True)


SERVE_STREAMS = 16
SERVE_BLOCK = 16_000_000       # 1 s at 16 Msps
SERVE_NBINS = 512
SERVE_METRIC = "serving: aggregate Msamples/s of 16 concurrent streams (1 s blocks), p50/p99 block latency"


def serve_streams(seed=4):
    """The 16 stream descriptions: DM log-uniform in [0.5, 200], period
    uniform in [2 ms, 2 s], FFT length the smallest power of two in
    [2^16, 2^24] whose half holds the smear's discard (2^24 otherwise),
    with the geometry from the library (pond_geometry)."""
    import numpy as np
    import paper_1503_01405_amd as P
    rng = np.random.default_rng(seed)
    out = []
    for i in range(SERVE_STREAMS):
        dm = float(np.exp(rng.uniform(np.log(0.5), np.log(200.0))))
        period = float(rng.uniform(2e-3, 2.0))
        n = 1 << 16
        while n < (1 << 24):
            g = P.pond_geometry(F0, BW, dm, n)
            if g is not None and g[1] <= n // 2:
                break
            n *= 2
        out.append(dict(dm=round(dm, 3), period_s=round(period, 6), nfft=n))
    return out


def serve_bytes(streams, blocks_per_stream, elem):
    """Pass-model bytes of every overlap-save block the streams complete
    (hop from the library's geometry)."""
    import paper_1503_01405_amd as P
    total = 0
    for s in streams:
        hop = P.pond_geometry(F0, BW, s["dm"], s["nfft"])[2]
        nsamp = blocks_per_stream * SERVE_BLOCK
        nb = 0 if nsamp < s["nfft"] else (nsamp - s["nfft"]) // hop + 1
        total += nb * s["nfft"] * (2 + 4 * elem)
    return total


def main_serve(args):
    import numpy as np
    import torch
    import paper_1503_01405_amd as P
    import synth

    form = [f for f in args.forms.split(",") if f and f != "fp32"] or ["fp32"]
    form = "half" if "half" in form else form[0]
    torch.cuda.init()
    streams = serve_streams()
    pool = []
    t = time.perf_counter()
    for k in range(4):
        h = torch.empty(2 * SERVE_BLOCK, dtype=torch.int8, pin_memory=True)
        h.numpy()[:] = synth.white_stream_int8(60 + k, SERVE_BLOCK)
        pool.append(h)
    log(f"generated 4 pinned 1 s blocks in {time.perf_counter() - t:.1f} s; streams {streams}")

    def open_all(srv):
        ids = []
        for s in streams:
            d = P.stream_desc(F0, BW, s["dm"], s["nfft"], SERVE_NBINS, s["period_s"], SERVE_BLOCK, SERVE_BLOCK, form)
            i = P.pond_server_open(srv, d)
            if i < 0:
                raise RuntimeError(f"stream {s} not admitted: {i}")
            ids.append(i)
        return ids

    # paced: each stream's block k arrives at phase + k s + Exp(20 ms)
    rng = np.random.default_rng(11)
    secs = args.serve_seconds
    arrivals = sorted((float(rng.uniform(0, 1)) + k + float(rng.exponential(0.02)), i, k)
                      for i in range(SERVE_STREAMS) for k in range(secs))
    srv = P.pond_server_create(200 << 30, 64)
    ids = open_all(srv)
    done = []
    t0 = time.perf_counter()
    for ta, i, k in arrivals:
        while time.perf_counter() - t0 < ta:
            done += P.pond_server_poll(srv)
            time.sleep(1e-4)
        if P.pond_server_submit(srv, ids[i], pool[(i + k) % 4], SERVE_BLOCK) < 0:
            raise RuntimeError("submit failed")
        done += P.pond_server_poll(srv)
    while True:
        got = P.pond_server_poll(srv, wait=True)
        if not got:
            break
        done += got
    for i in ids:
        P.pond_server_close(srv, i)
    P.pond_server_destroy(srv)
    lat = np.array([c["latency_us"] for c in done]) / 1e3
    dev = np.array([c["device_us"] for c in done]) / 1e3
    log(f"paced: {len(done)} blocks, latency p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms")

    # saturated: every block queued at once
    nblk = args.serve_burst_blocks
    srv = P.pond_server_create(200 << 30, 64)
    ids = open_all(srv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nblk):
        for j, i in enumerate(ids):
            if P.pond_server_submit(srv, i, pool[(j + k) % 4], SERVE_BLOCK) < 0:
                raise RuntimeError("submit failed")
    nb = 0
    while True:
        got = P.pond_server_poll(srv, 256, wait=True)
        if not got:
            break
        nb += len(got)
    wall = time.perf_counter() - t0
    for i in ids:
        P.pond_server_close(srv, i)
    P.pond_server_destroy(srv)
    total = SERVE_STREAMS * nblk * SERVE_BLOCK
    value = total / wall / 1e6
    elem = 8 if form == "fp32" else 4
    algo = serve_bytes(streams, nblk, elem)
    out = {
        "metric": SERVE_METRIC, "value": round(value, 1), "unit": "Msamples/s", "n_gpus": 1,
        "steps": nblk, "warmup": 0, "ms_per_step": round(wall * 1e3 / nblk, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"mixed": "f16 (matrix-core DFT) / f32 accumulate", "mixed_valu": "f16-storage/f32",
                  "half": "f16 (packed VALU) / f32 detect+fold",
                  "fp32": "f32"}[form],
        "data": "synthetic",
        "config": {"workload": "16 streams, DM log-uniform 0.5-200, P uniform 2 ms-2 s, nfft 2^16-2^24 by smear, "
                               "1 s int8 blocks from pinned host memory, 512 bins, 1 s subints",
                   "streams": streams, "form": form},
        "xrealtime_aggregate": round(value / 16.0, 1),
        "burst": {"blocks": SERVE_STREAMS * nblk, "seconds_of_data": SERVE_STREAMS * nblk, "wall_s": round(wall, 3)},
        "paced": {"seconds": secs, "blocks": len(done), "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                  "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                  "latency_ms_max": round(float(lat.max()), 3),
                  "device_ms_p50": round(float(np.percentile(dev, 50)), 3)},
        "roofline": dict(bound="hbm", kernel="whole burst (pass model)", achieved=round(algo / wall / 1e9, 1),
                         peak=HBM_PEAK_GBS, unit="GB/s", frac=round(algo / wall / 1e9 / HBM_PEAK_GBS, 4),
                         traffic=None),
    }
    print(json.dumps(out), flush=True)


AID_NCHAN, AID_NINT = 1024, 4
AID_METRIC = "AID Msamples/s filterbank+incoherent dedispersion+fold at DM 50 (1024 ch, 256 us)"


def aid_cpu_baseline(iq_np):
    """The oracle's AID path, as it stands, on the first 2^28 samples."""
    import oracle as O
    n = 1 << 28
    t0 = time.perf_counter()
    O.aid_run(iq_np[:2 * n], F0, BW, DM, AID_NCHAN, AID_NINT, NBINS, PERIOD)
    dt = time.perf_counter() - t0
    return dict(value=round(n / dt / 1e6, 3), unit="Msamples/s", cores=1, kind="oracle", **host_cpu(),
                sample=f"first {n} samples ({n / 16e6:.1f} s) of the same stream, {dt:.1f} s of CPU work (numpy FFTs, one thread)")


def main_aid(args):
    import torch
    import paper_1503_01405_amd as P
    import synth

    t = time.perf_counter()
    iq = synth.pulsed_stream_int8(SEED, NSAMP)
    log(f"generated {NSAMP} samples in {time.perf_counter() - t:.1f} s")
    x = torch.from_numpy(iq).to("cuda:0")
    h = P.pond_aid_create(F0, BW, DM, AID_NCHAN, AID_NINT, NBINS, PERIOD)
    geo = P.pond_aid_geometry(h, NSAMP)
    prof = torch.empty(NBINS, device="cuda:0")
    ser = torch.empty(geo["n_series"], device="cuda:0")
    stream = torch.cuda.current_stream()

    def step():
        n = P.pond_aid_run(h, x, NSAMP, prof, ser, ser.numel(), stream)
        if n != geo["n_series"]:
            raise RuntimeError(f"pond_aid_run returned {n}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = max((time.perf_counter() - t0) / args.steps * 1e3, ev0.elapsed_time(ev1) / args.steps)
    P.pond_aid_destroy(h)
    value = NSAMP / (ms / 1e3) / 1e6
    # bytes the two passes must move: int8 input, the integrated
    # filterbank written and read once, the series written
    algo = NSAMP * 2 + 2 * geo["n_spectra"] * AID_NCHAN * 4 + geo["n_series"] * 4
    out = {
        "metric": AID_METRIC, "value": round(value, 1), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "60 s 16 Msps int8 I/Q at 326.5 MHz, DM 50, 1024-channel filterbank, 4 spectra per "
                               "sample, 1024 bins", "nsamp": NSAMP, "nchan": AID_NCHAN, "nint": AID_NINT,
                   "n_series": geo["n_series"], "d_min": geo["d_min"], "d_max": geo["d_max"]},
        "xrealtime": round(value / 16.0, 1),
        "roofline": dict(bound="hbm", kernel="whole step (both passes)", achieved=round(algo / (ms / 1e3) / 1e9, 1),
                         peak=HBM_PEAK_GBS, unit="GB/s", frac=round(algo / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                         traffic=None, algorithmic_bytes_per_step=algo),
    }
    if not args.no_cpu_baseline:
        del x
        torch.cuda.empty_cache()
        out["cpu_baseline"] = aid_cpu_baseline(iq)
    print(json.dumps(out), flush=True)


REAL_NSAMP = 2 * NSAMP          # real samples, 60 s at 32 Msps
REAL_NFFT = 2 * NFFT            # real block length
REAL_SUBINT = 2 * SUBINT        # 10 s of real outputs
REAL_DECIM = 2 * DECIM          # 1 us
REAL_METRIC = "Msamples/s (real) dedispersed+folded at DM 50, real two-channel input"


def real_algorithmic_bytes(kernel, blocks, elem, n, hop_e, n1):
    """Per kernel slot of the real path, for `blocks` blocks of n packed
    elements: int8 A/B pairs (4 B per element) read once; the middle pass
    reads and writes the block once (rows up to 2^13: one fused kernel;
    longer rows: forward rows, split, inverse rows, three times); the
    inverse columns read it once and write the series."""
    if kernel == "k1_unpack_colfft":
        return blocks * n * (4 + elem)
    if kernel == "k2_row":
        return blocks * n * (2 if n1 <= 1 << 13 else 6) * elem
    if kernel == "k3_colinv_detect_fold":
        return blocks * (n * elem + hop_e // 16 * 4)
    return 0


def real_cpu_baseline(raw_np, sideband, nblocks):
    """The oracle's real path, as it stands, on the first `nblocks` blocks."""
    import oracle as O
    g = O.plan_geometry(F0, BW, DM, NFFT)
    n = 2 * g["hop"] * (nblocks - 1) + REAL_NFFT
    t0 = time.perf_counter()
    r = O.run_real(raw_np[:2 * n], F0, BW, DM, NFFT, NBINS, PERIOD, sideband=sideband, decim=REAL_DECIM)
    dt = time.perf_counter() - t0
    return dict(value=round(r["n_out"] / dt / 1e6, 3), unit="Msamples/s", cores=1, kind="oracle", **host_cpu(),
                sample=f"first {nblocks} blocks ({n} real samples) of the same stream, {dt:.1f} s of CPU work "
                       f"(scipy real FFTs, one thread)")


def main_real(args):
    import torch
    import paper_1503_01405_amd as P
    import synth

    t = time.perf_counter()
    # A and B: the I and Q draws of the generator at 32 Msps, each with half
    # the noise power, so that A + B has the complex recipe's component power
    raw = synth.pulsed_stream_int8(SEED, REAL_NSAMP, fs_hz=2 * BW * 1e6, sigma=synth.SIGMA / 2 ** 0.5)
    log(f"generated {REAL_NSAMP} real samples in {time.perf_counter() - t:.1f} s")
    x = torch.from_numpy(raw).to("cuda:0")
    forms = [f for f in args.forms.split(",") if f in ("fp32", "mixed_valu")] or ["fp32", "mixed_valu"]
    res = {}
    for f in forms:
        plan = P.Plan(F0, BW, DM, REAL_NFFT, NBINS, PERIOD, precision=f, subint_nsamp=REAL_SUBINT,
                      decim=REAL_DECIM, sideband="lsb")
        info = plan.info()
        nprof, nout = P.pond_real_expect(plan.handle, REAL_NSAMP, REAL_SUBINT)
        prof = torch.empty((nprof + 1, NBINS), dtype=torch.float32, device=x.device)
        ser = torch.empty(nout // REAL_DECIM, dtype=torch.float32, device=x.device)
        stream = torch.cuda.current_stream()

        def step():
            r, ns = P.pond_real_dedisperse(plan.handle, x, REAL_NSAMP, REAL_SUBINT, prof, nprof, REAL_DECIM,
                                           ser, ser.numel(), stream)
            if r != nprof or ns != ser.numel():
                raise RuntimeError(f"unexpected call result {r} {ns}")
            r, _ = P.pond_real_dedisperse(plan.handle, None, 0, REAL_SUBINT, prof[nprof:], 1, REAL_DECIM,
                                          None, 0, stream)
            if r != 1:
                raise RuntimeError(f"flush returned {r}")

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = max((time.perf_counter() - t0) / args.steps * 1e3, ev0.elapsed_time(ev1) / args.steps)
        P.pond_plan_set_timing(plan.handle, True)  # per-kernel times from a second pass
        for _ in range(args.steps):
            step()
        kt = P.pond_plan_kernel_times(plan.handle)
        plan.close()
        res[f] = dict(ms=ms, outputs=nout, kernels=kt, info=info)
        log(f"{f}: {ms:.3f} ms/step  kernels {kt}")
    head = "mixed_valu" if "mixed_valu" in res else forms[0]
    h = res[head]
    value = h["outputs"] / (h["ms"] / 1e3) / 1e6
    elem = 8 if head == "fp32" else 4
    kt = h["kernels"]
    dom = max(kt, key=lambda k: kt[k][0])
    ms, launches, blocks = kt[dom]
    n_e, hop_e = REAL_NFFT // 2, h["info"]["hop"] // 2
    algo = real_algorithmic_bytes(dom, blocks, elem, n_e, hop_e, h["info"]["n1"])
    achieved = algo / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    out = {
        "metric": REAL_METRIC, "value": round(value, 2), "unit": "Msamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(h["ms"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"mixed_valu": "f16-storage/f32", "fp32": "f32"}[head], "data": "synthetic",
        "config": {"workload": "60 s of 32 Msps real int8 A/B channel pairs at 326.5 MHz (lower sideband), DM 50, "
                               "real nfft 2^24, 1024 bins per 10 s subint, 1 us series",
                   "nsamp_real": REAL_NSAMP, "nfft_real": REAL_NFFT, "dm": DM, "nbins": NBINS,
                   "period_s": PERIOD, "subint_real": REAL_SUBINT, "decim_real": REAL_DECIM,
                   "valid_outputs_real": h["outputs"], "form": head},
        "xrealtime": round(value / 32.0, 1),
        "forms": {f: dict(value=round(r["outputs"] / (r["ms"] / 1e3) / 1e6, 2), ms_per_step=round(r["ms"], 3),
                          kernel_ms_per_step={k: round(kv[0] / args.steps, 4) for k, kv in r["kernels"].items()})
                  for f, r in res.items()},
        "roofline": dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                         copy_achievable=round(copy_bandwidth(), 1),
                         algorithmic_bytes_per_launch=int(algo / max(launches, 1)),
                         avg_launch_us=round(ms / max(launches, 1) * 1e3, 2)),
    }
    if not args.no_cpu_baseline:
        del x
        torch.cuda.empty_cache()
        out["cpu_baseline"] = real_cpu_baseline(raw, "lsb", min(args.cpu_blocks, 24))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="fp32,mixed_valu,mixed,half,bf16")
    ap.add_argument("--cpu-blocks", type=int, default=80,
                    help="blocks of the stream the CPU oracle baseline processes (about 15 s on 16 cores)")
    ap.add_argument("--graph", action="store_true",
                    help="also time the step captured once into a HIP graph and replayed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["dm50", "search", "serve", "aid", "real"], default="dm50",
                    help="dm50: the single-DM production stream (default); search: the 128-trial DM search; "
                         "serve: the 16-stream serving loop; aid: the filterbank mode; real: the real "
                         "two-channel input path")
    ap.add_argument("--serve-seconds", type=int, default=8, help="paced serving run length (s)")
    ap.add_argument("--serve-burst-blocks", type=int, default=8, help="1 s blocks per stream in the saturated run")
    ap.add_argument("--max-batch", type=int, default=0,
                    help="blocks per launch (default: the library's autotuner picks them)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the path shards by block range across GPUs as described in the design notes",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "search":
        main_search(args)
        return
    if args.workload == "serve":
        main_serve(args)
        return
    if args.workload == "aid":
        main_aid(args)
        return
    if args.workload == "real":
        main_real(args)
        return

    import numpy as np
    import torch
    import synth

    t = time.perf_counter()
    iq = synth.pulsed_stream_int8(SEED, NSAMP)
    log(f"generated {NSAMP} samples in {time.perf_counter() - t:.1f} s")
    x = torch.from_numpy(iq).to("cuda:0")
    torch.cuda.synchronize()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n} bytes device-to-device")
        del src, dst

    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for f in forms:
        res[f] = run_form(f, x, args.steps, args.warmup, graph=args.graph, max_batch=args.max_batch)
        log(f"{f}: {res[f]['ms_per_step']:.3f} ms/step  kernels {res[f]['kernels']}")

    # headline: the fastest float16 form (bfloat16 storage is a reported
    # variant only, not held to the 1e-4 accuracy)
    mixed = [f for f in res if f not in ("fp32", "bf16")]
    head = min(mixed, key=lambda f: res[f]["ms_per_step"]) if mixed else forms[0]
    h = res[head]
    hop = h["info"]["hop"]
    value = h["outputs"] / (h["ms_per_step"] / 1e3) / 1e6

    # roofline of the kernel that takes the most time in the headline form
    elem = 8 if head == "fp32" else 4
    kt = h["kernels"]
    dom = max(kt, key=lambda k: kt[k][0])
    ms, launches, blocks = kt[dom]
    algo = algorithmic_bytes(dom, blocks, elem, NFFT, hop)
    achieved = algo / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    avg_s = ms / 1e3 / max(launches, 1)
    per_block = measured_traffic(dom, head, h["info"]["max_batch"])
    bpl = blocks / max(launches, 1)
    meas = int(sum(per_block) * bpl) if per_block else None
    copy_gbs = copy_bandwidth()
    log(f"library streaming copy: {copy_gbs:.0f} GB/s")
    roof = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                copy_achievable=round(copy_gbs, 1), frac_of_copy=round(achieved / copy_gbs, 4),
                traffic=round(meas / avg_s / 1e9, 1) if meas else None,
                traffic_bytes_per_launch=meas,
                algorithmic_bytes_per_launch=int(algo / max(launches, 1)),
                avg_launch_us=round(avg_s * 1e6, 2), blocks_per_launch=round(blocks / max(launches, 1), 3))

    forms_out = {}
    for f, r in res.items():
        v = r["outputs"] / (r["ms_per_step"] / 1e3) / 1e6
        tu = r["tune"]
        forms_out[f] = dict(value=round(v, 2), xrealtime=round(v / 16.0, 1), ms_per_step=round(r["ms_per_step"], 3),
                            kernel_ms_per_step={k: round(kv[0] / args.steps, 4) for k, kv in r["kernels"].items()},
                            blocks_per_launch=r["info"]["max_batch"])
        if tu:
            forms_out[f]["autotune"] = dict(batch=tu["batch"], ms_per_block=round(tu["ms_per_block"], 4),
                                            default_batch=tu["default_batch"],
                                            default_ms_per_block=round(tu["default_ms_per_block"], 4),
                                            from_cache=tu["from_cache"])
        if "graph_ms_per_step" in r:
            forms_out[f]["graph_ms_per_step"] = round(r["graph_ms_per_step"], 3)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f16 (matrix-core DFT) / f32 accumulate", "mixed_valu": "f16-storage/f32",
                  "half": "f16 (packed VALU) / f32 detect+fold", "bf16": "bf16-storage/f32",
                  "fp32": "f32"}[head],
        "data": "synthetic",
        "config": {"workload": "60 s 16 Msps int8 I/Q at 326.5 MHz, DM 50, nfft 2^23 (2^22 discarded), "
                               "1024 bins per 10 s subint, 1 us series",
                   "nsamp": NSAMP, "nfft": NFFT, "dm": DM, "nbins": NBINS, "period_s": PERIOD,
                   "subint_outputs": SUBINT, "decim": DECIM, "valid_outputs": h["outputs"],
                   "form": head},
        "xrealtime": round(value / 16.0, 1),
        "forms": forms_out,
        "roofline": roof,
    }
    if "fp32" in res:
        for f in mixed:
            out[f"speedup_{f}_vs_fp32"] = round(res["fp32"]["ms_per_step"] / res[f]["ms_per_step"], 3)
    if not args.no_cpu_baseline:
        del x
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(iq, args.cpu_blocks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
