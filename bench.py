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


def kernel_source_hash():
    """sha256[:16] over the HIP/C++ sources of the library (as recorded in
    the committed rocprofv3 summaries)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1503_01405_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_prefix):
    """HBM bytes per dispatch of a kernel from the committed counter summary,
    or None if the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_bytes_dm50_nfft2e23_mixed.txt")
    if not os.path.exists(path):
        return None
    src = None
    with open(path) as fh:
        lines = fh.read().splitlines()
    for ln in lines:
        if ln.startswith("kernel source sha256[:16]:"):
            src = ln.rsplit(":", 1)[1].strip()
    if src != kernel_source_hash():
        return None
    for ln in lines:
        if ln.startswith("TRAFFIC ") and kernel_prefix in ln and "__half2" in ln:
            kv = dict(t.split("=") for t in ln.split() if "=" in t)
            return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def run_form(precision, x, steps, warmup, graph=False):
    import torch
    import paper_1503_01405_amd as P

    plan = P.Plan(F0, BW, DM, NFFT, NBINS, PERIOD, precision=precision, subint_nsamp=SUBINT, decim=DECIM)
    info = plan.info()
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
    P.pond_plan_set_timing(plan.handle, True)
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
    kt = P.pond_plan_kernel_times(plan.handle)
    P.pond_plan_set_timing(plan.handle, False)
    ms = max(wall, ev_ms)
    res = dict(ms_per_step=ms, ms_events=ev_ms, ms_wall=wall, outputs=nout, kernels=kt, info=info)
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
    return dict(value=round(msps, 3), unit="Msamples/s", cores=workers, kind="oracle",
                sample=f"first {nblocks} of 227 overlap-save blocks ({r['n_out']} outputs, "
                       f"{r['n_out'] / 16e6:.2f} s of data) of the same stream, {dt:.1f} s of CPU work",
                xrealtime=round(msps / 16.0, 3))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--forms", default="fp32,mixed_valu,mixed")
    ap.add_argument("--cpu-blocks", type=int, default=16)
    ap.add_argument("--graph", action="store_true",
                    help="also time the step captured once into a HIP graph and replayed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a known-size "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the path shards by block range across GPUs as described in the design notes",
              file=sys.stderr)
        sys.exit(2)

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
        res[f] = run_form(f, x, args.steps, args.warmup, graph=args.graph)
        log(f"{f}: {res[f]['ms_per_step']:.3f} ms/step  kernels {res[f]['kernels']}")

    head = "mixed" if "mixed" in res else forms[0]
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
    meas = measured_traffic(dom) if head == "mixed" else None
    roof = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=round(meas / avg_s / 1e9, 1) if meas else None,
                traffic_bytes_per_launch=meas,
                algorithmic_bytes_per_launch=int(algo / max(launches, 1)),
                avg_launch_us=round(avg_s * 1e6, 2), blocks_per_launch=round(blocks / max(launches, 1), 3))

    forms_out = {}
    for f, r in res.items():
        v = r["outputs"] / (r["ms_per_step"] / 1e3) / 1e6
        forms_out[f] = dict(value=round(v, 2), xrealtime=round(v / 16.0, 1), ms_per_step=round(r["ms_per_step"], 3),
                            kernel_ms_per_step={k: round(kv[0] / args.steps, 4) for k, kv in r["kernels"].items()})
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
    if "mixed" in res and "fp32" in res:
        out["speedup_mixed_vs_fp32"] = round(res["fp32"]["ms_per_step"] / res["mixed"]["ms_per_step"], 3)
    if not args.no_cpu_baseline:
        del x
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(iq, args.cpu_blocks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
