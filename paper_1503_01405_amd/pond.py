"""ctypes binding of libpond.so (include/pond.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are passed as torch CUDA tensors (their data_ptr())
and streams as torch.cuda.Stream objects (their cuda_stream handle).  If
the library has not been built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpond.so")

POND_OK = 0
POND_EINVAL = -1
POND_ENOMEM = -2
POND_EDEVICE = -3
POND_EBUSY = -4
POND_ECANCELED = -5

POND_TICKET_ADMITTED = -1
POND_STREAM_WAITING = 0
POND_STREAM_OPEN = 1
POND_STREAM_CLOSED = 2

POND_FP32 = 0
POND_MIXED = 1
POND_MIXED_VALU = 2
POND_HALF = 3
POND_BF16 = 4
FORMS = {"fp32": POND_FP32, "mixed": POND_MIXED, "mixed_valu": POND_MIXED_VALU, "half": POND_HALF,
         "bf16": POND_BF16}

POND_STATUS_NONFINITE = 1
POND_STATUS_RANGE = 2

POND_BATCH_AUTOTUNE = -1

POND_INPUT_COMPLEX = 0
POND_INPUT_REAL_LSB = 1
POND_INPUT_REAL_USB = 2
POND_LSB = 0
POND_USB = 1
SIDEBANDS = {"lsb": POND_LSB, "usb": POND_USB}

EXPORTS = (
    "pond_plan_create", "pond_plan_create_ex", "pond_create_status",
    "pond_dedisperse_fold", "pond_dedisperse_series", "pond_plan_query",
    "pond_plan_expect", "pond_plan_destroy", "pond_strerror",
    "pond_plan_set_timing", "pond_plan_kernel_times", "pond_plan_set_taper",
    "pond_search_create", "pond_search_run", "pond_search_trial", "pond_search_destroy",
    "pond_search_create_ex", "pond_search_autotune",
    "pond_server_create", "pond_server_stream_bytes", "pond_server_open", "pond_server_submit",
    "pond_server_poll", "pond_server_take_profiles", "pond_server_close", "pond_server_query",
    "pond_server_destroy", "pond_server_stream_state",
    "pond_aid_create", "pond_aid_geometry", "pond_aid_run", "pond_aid_destroy",
    "pond_real_plan_create", "pond_real_dedisperse", "pond_real_expect",
    "pond_copy_device", "pond_geometry", "pond_dedisperse_segment_noalloc", "pond_plan_autotune",
)
KERNEL_NAMES = ("k1_unpack_colfft", "k2_row", "k3_colinv_detect_fold", "fold_reduce", "fold_finalize")


class PondError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = int(code)
        msg = _lib.pond_strerror(int(code)).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class pond_info(ctypes.Structure):
    _fields_ = [
        ("nfft", ctypes.c_int64), ("n_front", ctypes.c_int64),
        ("discard", ctypes.c_int64), ("hop", ctypes.c_int64),
        ("n1", ctypes.c_int64), ("n2", ctypes.c_int64),
        ("samples_in", ctypes.c_int64), ("outputs_done", ctypes.c_int64),
        ("max_batch", ctypes.c_int64),
        ("fs_hz", ctypes.c_double), ("delta_lo_s", ctypes.c_double),
        ("delta_hi_s", ctypes.c_double), ("inv_pfs", ctypes.c_double),
        ("nbins", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("status", ctypes.c_uint32), ("input_kind", ctypes.c_int32),
        ("power_gain", ctypes.c_double),
    ]


class pond_kernel_times(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 5), ("launches", ctypes.c_int64 * 5),
                ("blocks", ctypes.c_int64 * 5)]


class pond_stream_desc(ctypes.Structure):
    _fields_ = [
        ("f0_mhz", ctypes.c_double), ("bw_mhz", ctypes.c_double), ("dm", ctypes.c_double),
        ("period_s", ctypes.c_double), ("nfft", ctypes.c_int64), ("subint_nsamp", ctypes.c_int64),
        ("max_block_nsamp", ctypes.c_int64), ("nbins", ctypes.c_int32), ("precision", ctypes.c_int32),
    ]


class pond_completion(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_int64), ("stream", ctypes.c_int32), ("status", ctypes.c_int32),
        ("n_profiles", ctypes.c_int64), ("latency_us", ctypes.c_double), ("device_us", ctypes.c_double),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_1503_01405_amd/build.py")
    # torch first: its HIP runtime (soname libamdhip64.so.7) then satisfies
    # the library's dependency, so device pointers, streams and graphs of
    # both live in ONE runtime.  Loaded the other way round, the process
    # would hold two HIP runtimes and torch would find no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.pond_plan_create.argtypes = [dbl, dbl, dbl, i64, i32, dbl]
    lib.pond_plan_create.restype = P
    lib.pond_plan_create_ex.argtypes = [dbl, dbl, dbl, i64, i32, dbl, i32, i32]
    lib.pond_plan_create_ex.restype = P
    lib.pond_create_status.argtypes = []
    lib.pond_create_status.restype = i32
    lib.pond_dedisperse_fold.argtypes = [P, P, i64, i64, P, i64, P]
    lib.pond_dedisperse_fold.restype = i64
    lib.pond_dedisperse_series.argtypes = [P, P, i64, i64, P, i64, i32, P, i64,
                                           ctypes.POINTER(i64), P]
    lib.pond_dedisperse_series.restype = i64
    lib.pond_plan_query.argtypes = [P, ctypes.POINTER(pond_info)]
    lib.pond_plan_query.restype = i32
    lib.pond_plan_autotune.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    lib.pond_plan_autotune.restype = i32
    lib.pond_plan_expect.argtypes = [P, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.pond_plan_expect.restype = i32
    lib.pond_plan_destroy.argtypes = [P]
    lib.pond_plan_destroy.restype = None
    lib.pond_plan_set_timing.argtypes = [P, i32]
    lib.pond_plan_set_timing.restype = i32
    lib.pond_plan_set_taper.argtypes = [P, dbl]
    lib.pond_plan_set_taper.restype = i32
    lib.pond_plan_kernel_times.argtypes = [P, ctypes.POINTER(pond_kernel_times)]
    lib.pond_plan_kernel_times.restype = i32
    lib.pond_search_create.argtypes = [dbl, dbl, ctypes.POINTER(dbl), i32, i32, dbl, i64, i64, i32]
    lib.pond_search_create.restype = P
    lib.pond_search_create_ex.argtypes = [dbl, dbl, ctypes.POINTER(dbl), i32, i32, dbl, i64, i64, i32, i32]
    lib.pond_search_create_ex.restype = P
    lib.pond_search_autotune.argtypes = [P, i64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    lib.pond_search_autotune.restype = i32
    lib.pond_search_run.argtypes = [P, P, i64, P, P]
    lib.pond_search_run.restype = i32
    lib.pond_search_trial.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.pond_search_trial.restype = i32
    lib.pond_search_destroy.argtypes = [P]
    lib.pond_search_destroy.restype = None
    lib.pond_server_create.argtypes = [i64, i32]
    lib.pond_server_create.restype = P
    lib.pond_server_stream_bytes.argtypes = [ctypes.POINTER(pond_stream_desc)]
    lib.pond_server_stream_bytes.restype = i64
    lib.pond_server_open.argtypes = [P, ctypes.POINTER(pond_stream_desc)]
    lib.pond_server_open.restype = i32
    lib.pond_server_submit.argtypes = [P, i32, P, i64]
    lib.pond_server_submit.restype = i64
    lib.pond_server_poll.argtypes = [P, ctypes.POINTER(pond_completion), i32, i32]
    lib.pond_server_poll.restype = i32
    lib.pond_server_take_profiles.argtypes = [P, i32, P, i64]
    lib.pond_server_take_profiles.restype = i64
    lib.pond_server_close.argtypes = [P, i32]
    lib.pond_server_close.restype = i32
    lib.pond_dedisperse_segment_noalloc.argtypes = [dbl, dbl, dbl, i64, i32, dbl, i32, P, i64, i32, P, P, i64, P]
    lib.pond_dedisperse_segment_noalloc.restype = i64
    lib.pond_geometry.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, i64,
                                  ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.pond_geometry.restype = i32
    lib.pond_server_stream_state.argtypes = [P, i32]
    lib.pond_server_stream_state.restype = i32
    lib.pond_server_query.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                      ctypes.POINTER(i64)]
    lib.pond_server_query.restype = i32
    lib.pond_server_destroy.argtypes = [P]
    lib.pond_server_destroy.restype = None
    lib.pond_aid_create.argtypes = [dbl, dbl, dbl, i32, i32, i32, dbl]
    lib.pond_aid_create.restype = P
    lib.pond_aid_geometry.argtypes = [P, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                      ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.pond_aid_geometry.restype = i32
    lib.pond_aid_run.argtypes = [P, P, i64, P, P, i64, P]
    lib.pond_aid_run.restype = i64
    lib.pond_aid_destroy.argtypes = [P]
    lib.pond_aid_destroy.restype = None
    lib.pond_real_plan_create.argtypes = [dbl, dbl, dbl, i64, i32, dbl, i32, i32, i32]
    lib.pond_real_plan_create.restype = P
    lib.pond_real_dedisperse.argtypes = [P, P, i64, i64, P, i64, i32, P, i64, ctypes.POINTER(i64), P]
    lib.pond_real_dedisperse.restype = i64
    lib.pond_real_expect.argtypes = [P, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.pond_real_expect.restype = i32
    lib.pond_copy_device.argtypes = [P, P, i64, P]
    lib.pond_copy_device.restype = i32
    lib.pond_strerror.argtypes = [i64]
    lib.pond_strerror.restype = ctypes.c_char_p
    return lib


_lib = None
_lib = _load()


def lib():
    return _lib


def _ptr(t):
    """Device address of a tensor (or None/int)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------- C-ABI-named wrappers
def pond_plan_create(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, precision=POND_FP32, max_batch=0):
    """Create a plan; returns the opaque handle (int).  Raises PondError."""
    h = _lib.pond_plan_create_ex(float(f0_mhz), float(bw_mhz), float(dm), int(nfft), int(nbins),
                                 float(period_s), int(precision), int(max_batch))
    if not h:
        raise PondError(_lib.pond_create_status(), "pond_plan_create")
    return h


def pond_dedisperse_fold(plan, iq, nsamp, subint_nsamp, profiles, max_profiles, stream=None):
    return _lib.pond_dedisperse_fold(plan, _ptr(iq), int(nsamp), int(subint_nsamp), _ptr(profiles),
                                     int(max_profiles), _stream(stream))


def pond_dedisperse_series(plan, iq, nsamp, subint_nsamp, profiles, max_profiles, decim, series,
                           series_cap, stream=None):
    """Returns (profiles written or error code, series values written)."""
    n = ctypes.c_int64(0)
    r = _lib.pond_dedisperse_series(plan, _ptr(iq), int(nsamp), int(subint_nsamp), _ptr(profiles),
                                    int(max_profiles), int(decim), _ptr(series), int(series_cap),
                                    ctypes.byref(n), _stream(stream))
    return r, n.value


def pond_plan_query(plan):
    info = pond_info()
    r = _lib.pond_plan_query(plan, ctypes.byref(info))
    if r != POND_OK:
        raise PondError(r, "pond_plan_query")
    return {name: getattr(info, name) for name, _ in pond_info._fields_}


def pond_plan_autotune(plan):
    """The autotuner's choice for a plan created with POND_BATCH_AUTOTUNE:
    dict of batch, ms_per_block, default_batch, default_ms_per_block,
    from_cache."""
    b, d, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    t, td = ctypes.c_double(0), ctypes.c_double(0)
    r = _lib.pond_plan_autotune(plan, ctypes.byref(b), ctypes.byref(t), ctypes.byref(d), ctypes.byref(td),
                                ctypes.byref(c))
    if r != POND_OK:
        raise PondError(r, "pond_plan_autotune")
    return {"batch": b.value, "ms_per_block": t.value, "default_batch": d.value,
            "default_ms_per_block": td.value, "from_cache": bool(c.value)}


def pond_plan_expect(plan, nsamp, subint_nsamp):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    r = _lib.pond_plan_expect(plan, int(nsamp), int(subint_nsamp), ctypes.byref(a), ctypes.byref(b))
    if r != POND_OK:
        raise PondError(r, "pond_plan_expect")
    return a.value, b.value


def pond_plan_destroy(plan):
    _lib.pond_plan_destroy(plan)


def pond_plan_set_timing(plan, enable):
    r = _lib.pond_plan_set_timing(plan, int(bool(enable)))
    if r != POND_OK:
        raise PondError(r, "pond_plan_set_timing")


def pond_plan_kernel_times(plan):
    """{kernel name: (ms, launches, blocks)} since timing was enabled."""
    t = pond_kernel_times()
    r = _lib.pond_plan_kernel_times(plan, ctypes.byref(t))
    if r != POND_OK:
        raise PondError(r, "pond_plan_kernel_times")
    return {KERNEL_NAMES[i]: (t.ms[i], t.launches[i], t.blocks[i]) for i in range(5)}


def pond_plan_set_taper(plan, alpha):
    r = _lib.pond_plan_set_taper(plan, float(alpha))
    if r != POND_OK:
        raise PondError(r, "pond_plan_set_taper")


def pond_real_plan_create(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, precision=POND_FP32, max_batch=0,
                          sideband=POND_LSB):
    """Real two-channel input plan (nfft: real block length); raises PondError."""
    if isinstance(sideband, str):
        sideband = SIDEBANDS[sideband]
    h = _lib.pond_real_plan_create(float(f0_mhz), float(bw_mhz), float(dm), int(nfft), int(nbins),
                                   float(period_s), int(precision), int(max_batch), int(sideband))
    if not h:
        raise PondError(_lib.pond_create_status(), "pond_real_plan_create")
    return h


def pond_real_dedisperse(plan, raw, nsamp, subint_nsamp, profiles, max_profiles, decim=32, series=None,
                         series_cap=0, stream=None):
    """Returns (profiles written or error code, series values written)."""
    n = ctypes.c_int64(0)
    r = _lib.pond_real_dedisperse(plan, _ptr(raw), int(nsamp), int(subint_nsamp), _ptr(profiles),
                                  int(max_profiles), int(decim), _ptr(series), int(series_cap),
                                  ctypes.byref(n), _stream(stream))
    return r, n.value


def pond_real_expect(plan, nsamp, subint_nsamp):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    r = _lib.pond_real_expect(plan, int(nsamp), int(subint_nsamp), ctypes.byref(a), ctypes.byref(b))
    if r != POND_OK:
        raise PondError(r, "pond_real_expect")
    return a.value, b.value


def pond_copy_device(dst, src, nbytes, stream=None):
    """The library's streaming device copy (for bandwidth measurement)."""
    r = _lib.pond_copy_device(_ptr(dst), _ptr(src), int(nbytes), _stream(stream))
    if r != POND_OK:
        raise PondError(r, "pond_copy_device")


def pond_search_create(f0_mhz, bw_mhz, dms, nbins, period_s, nfft_min=1 << 20, nfft_max=1 << 23,
                       precision=POND_FP32, max_batch=None):
    """Create a DM-trial search; max_batch (None: pond_search_create's
    default) as for pond_search_create_ex, e.g. POND_BATCH_AUTOTUNE."""
    arr = (ctypes.c_double * len(dms))(*[float(d) for d in dms])
    if max_batch is None:
        h = _lib.pond_search_create(float(f0_mhz), float(bw_mhz), arr, len(dms), int(nbins), float(period_s),
                                    int(nfft_min), int(nfft_max), int(precision))
    else:
        h = _lib.pond_search_create_ex(float(f0_mhz), float(bw_mhz), arr, len(dms), int(nbins), float(period_s),
                                       int(nfft_min), int(nfft_max), int(precision), int(max_batch))
    if not h:
        raise PondError(POND_EINVAL, "pond_search_create")
    return h


def pond_search_autotune(search, nfft):
    """The autotuner's result for the search's length group of FFT length
    nfft (dict as pond_plan_autotune)."""
    b, d, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    t, td = ctypes.c_double(0), ctypes.c_double(0)
    r = _lib.pond_search_autotune(search, int(nfft), ctypes.byref(b), ctypes.byref(t), ctypes.byref(d),
                                  ctypes.byref(td), ctypes.byref(c))
    if r != POND_OK:
        raise PondError(r, "pond_search_autotune")
    return {"batch": b.value, "ms_per_block": t.value, "default_batch": d.value,
            "default_ms_per_block": td.value, "from_cache": bool(c.value)}


def pond_search_run(search, iq, nsamp, profiles, stream=None):
    return _lib.pond_search_run(search, _ptr(iq), int(nsamp), _ptr(profiles), _stream(stream))


def pond_search_trial(search, t):
    n, f, h = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    r = _lib.pond_search_trial(search, int(t), ctypes.byref(n), ctypes.byref(f), ctypes.byref(h))
    if r != POND_OK:
        raise PondError(r, "pond_search_trial")
    return n.value, f.value, h.value


def pond_search_destroy(search):
    _lib.pond_search_destroy(search)


def _desc(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, subint_nsamp, max_block_nsamp, precision):
    prec = FORMS.get(precision, precision)
    return pond_stream_desc(float(f0_mhz), float(bw_mhz), float(dm), float(period_s), int(nfft),
                            int(subint_nsamp), int(max_block_nsamp), int(nbins), int(prec))


def pond_server_create(hbm_budget_bytes, max_streams=64):
    h = _lib.pond_server_create(int(hbm_budget_bytes), int(max_streams))
    if not h:
        raise PondError(POND_EINVAL, "pond_server_create")
    return h


def pond_server_stream_bytes(desc):
    return _lib.pond_server_stream_bytes(ctypes.byref(desc))


def pond_server_open(server, desc):
    return _lib.pond_server_open(server, ctypes.byref(desc))


def pond_server_submit(server, stream, host_iq, nsamp):
    """host_iq: a CPU tensor or numpy int8 array (2*nsamp values) that stays
    alive and unmodified until the block is reported by poll."""
    ptr = host_iq.data_ptr() if hasattr(host_iq, "data_ptr") else host_iq.ctypes.data
    return _lib.pond_server_submit(server, int(stream), ptr, int(nsamp))


def pond_server_poll(server, max_out=64, wait=False):
    buf = (pond_completion * max_out)()
    n = _lib.pond_server_poll(server, buf, int(max_out), 1 if wait else 0)
    if n < 0:
        raise PondError(n, "pond_server_poll")
    return [dict(ticket=c.ticket, stream=c.stream, status=c.status, n_profiles=c.n_profiles,
                 latency_us=c.latency_us, device_us=c.device_us) for c in buf[:n]]


def pond_server_take_profiles(server, stream, nbins, max_profiles=1 << 20):
    import numpy as np
    out = np.empty((0, nbins), dtype=np.float32)
    while True:
        chunk = np.empty((4096, nbins), dtype=np.float32)
        n = _lib.pond_server_take_profiles(server, int(stream), chunk.ctypes.data, 4096)
        if n < 0:
            raise PondError(n, "pond_server_take_profiles")
        out = np.concatenate([out, chunk[:n]])
        if n < 4096 or out.shape[0] >= max_profiles:
            return out


def pond_server_close(server, stream):
    return _lib.pond_server_close(server, int(stream))


def pond_dedisperse_segment_noalloc(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, precision, iq, nsamp, decim,
                                    profile, series, series_cap, stream=None):
    """One resident segment through the whole path with no device
    allocation (the library's static scratch); returns the series count or
    a negative error code."""
    return _lib.pond_dedisperse_segment_noalloc(float(f0_mhz), float(bw_mhz), float(dm), int(nfft), int(nbins),
                                                float(period_s), int(precision), _ptr(iq), int(nsamp),
                                                int(decim), _ptr(profile), _ptr(series), int(series_cap),
                                                _stream(stream))


def pond_geometry(f0_mhz, bw_mhz, dm, nfft):
    """(n_front, discard, hop) of a plan with these arguments, or None if
    no plan can be made (hop would not be positive, or bad arguments)."""
    nf, d, h = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    r = _lib.pond_geometry(float(f0_mhz), float(bw_mhz), float(dm), int(nfft), ctypes.byref(nf), ctypes.byref(d),
                           ctypes.byref(h))
    return (nf.value, d.value, h.value) if r == POND_OK else None


def pond_server_stream_state(server, stream):
    return _lib.pond_server_stream_state(server, int(stream))


def pond_server_query(server):
    u, b, q = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    o = ctypes.c_int32(0)
    r = _lib.pond_server_query(server, ctypes.byref(u), ctypes.byref(b), ctypes.byref(o), ctypes.byref(q))
    if r != POND_OK:
        raise PondError(r, "pond_server_query")
    return dict(used_bytes=u.value, budget_bytes=b.value, open_streams=o.value, queued_blocks=q.value)


def pond_server_destroy(server):
    _lib.pond_server_destroy(server)


def pond_aid_create(f0_mhz, bw_mhz, dm, nchan, nint, nbins, period_s):
    h = _lib.pond_aid_create(float(f0_mhz), float(bw_mhz), float(dm), int(nchan), int(nint), int(nbins),
                             float(period_s))
    if not h:
        raise PondError(POND_EINVAL, "pond_aid_create")
    return h


def pond_aid_geometry(aid, nsamp):
    ns, no = ctypes.c_int64(0), ctypes.c_int64(0)
    dmin, dmax = ctypes.c_int32(0), ctypes.c_int32(0)
    ts = ctypes.c_double(0)
    r = _lib.pond_aid_geometry(aid, int(nsamp), ctypes.byref(ns), ctypes.byref(no), ctypes.byref(dmin),
                               ctypes.byref(dmax), ctypes.byref(ts))
    if r != POND_OK:
        raise PondError(r, "pond_aid_geometry")
    return dict(n_spectra=ns.value, n_series=no.value, d_min=dmin.value, d_max=dmax.value, t_s=ts.value)


def pond_aid_run(aid, iq, nsamp, profile, series=None, series_cap=0, stream=None):
    return _lib.pond_aid_run(aid, _ptr(iq), int(nsamp), _ptr(profile), _ptr(series), int(series_cap),
                             _stream(stream))


def pond_aid_destroy(aid):
    _lib.pond_aid_destroy(aid)


# ------------------------------------------------------- convenience class
class Plan:
    """A dedispersion + fold plan on the current torch device.

    ``process(iq)`` appends a device int8 tensor and returns the profiles
    completed by the call (float32, [k, nbins]) and, if asked, the new
    decimated series values; ``flush()`` ends the stream and returns the
    open sub-integration's profile.  Output tensors are allocated with torch
    on the plan's device.  With ``sideband`` ("lsb" or "usb") the plan takes
    the real two-channel input (int8 A/B pairs) and nfft, subint_nsamp and
    decim count real samples.
    """

    def __init__(self, f0_mhz, bw_mhz, dm, nfft, nbins, period_s, precision="fp32",
                 max_batch=0, subint_nsamp=0, decim=None, taper_alpha=0.0, sideband=None):
        prec = FORMS.get(precision, precision)
        self.real = sideband is not None
        if self.real:
            self.handle = pond_real_plan_create(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, prec,
                                                max_batch, sideband)
        else:
            self.handle = pond_plan_create(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, prec, max_batch)
        if taper_alpha:
            pond_plan_set_taper(self.handle, taper_alpha)
        self.nbins = int(nbins)
        self.subint = int(subint_nsamp)
        self.decim = int(decim) if decim is not None else (32 if self.real else 16)

    def info(self):
        return pond_plan_query(self.handle)

    def autotune(self):
        """The autotuner's result (plans created with max_batch=POND_BATCH_AUTOTUNE)."""
        return pond_plan_autotune(self.handle)

    def _expect(self, nsamp):
        return (pond_real_expect if self.real else pond_plan_expect)(self.handle, nsamp, self.subint)

    def _call(self, iq, nsamp, prof, nprof, ser, stream):
        if self.real:
            return pond_real_dedisperse(self.handle, iq, nsamp, self.subint, prof, nprof, self.decim,
                                        ser, ser.numel() if ser is not None else 0, stream)
        if ser is not None:
            return pond_dedisperse_series(self.handle, iq, nsamp, self.subint, prof, nprof,
                                          self.decim, ser, ser.numel(), stream)
        return pond_dedisperse_fold(self.handle, iq, nsamp, self.subint, prof, nprof, stream), 0

    def process(self, iq, want_series=True, stream=None):
        import torch
        nsamp = iq.numel() // 2
        if nsamp == 0:   # a NULL/0 call would end the stream
            empty = torch.empty((0, self.nbins), dtype=torch.float32, device=iq.device)
            return empty, (torch.empty(0, dtype=torch.float32, device=iq.device) if want_series else None)
        nprof, nout = self._expect(nsamp)
        prof = torch.empty((max(nprof, 0), self.nbins), dtype=torch.float32, device=iq.device)
        ser = torch.empty(nout // self.decim, dtype=torch.float32, device=iq.device) if want_series else None
        r, ns = self._call(iq, nsamp, prof, nprof, ser, stream)
        if r < 0:
            raise PondError(r, "process")
        return prof[:r], (ser[:ns] if ser is not None else None)

    def flush(self, device=None, stream=None):
        import torch
        nprof, _ = self._expect(0)
        prof = torch.empty((nprof, self.nbins), dtype=torch.float32,
                           device=device if device is not None else torch.device("cuda"))
        r, _ = self._call(None, 0, prof, nprof, None, stream)
        if r < 0:
            raise PondError(r, "flush")
        return prof[:r]

    def close(self):
        if self.handle:
            pond_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
