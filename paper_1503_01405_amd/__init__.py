"""MI355X-native overlap-save coherent dedispersion and folding of complex
baseband voltages (the pulsar mode of PONDER, arXiv:1503.01405).

The compute path lives in libpond.so (HIP kernels for gfx950 behind the C
ABI of include/pond.h); this package is its ctypes binding.
"""
from .pond import (POND_EBUSY, POND_EDEVICE, POND_EINVAL, POND_ENOMEM, FORMS, POND_FP32, POND_HALF, POND_MIXED, POND_MIXED_VALU,  # noqa: F401
                   POND_OK, POND_STATUS_NONFINITE, POND_STATUS_RANGE, Plan, PondError,
                   pond_dedisperse_fold, pond_dedisperse_series, pond_plan_create,
                   pond_plan_destroy, pond_plan_expect, pond_plan_kernel_times,
                   pond_plan_query, pond_plan_set_taper, pond_plan_set_timing, pond_search_create, pond_search_destroy,
                   pond_search_run, pond_search_trial, pond_server_close, pond_server_create,
                   pond_server_destroy, pond_server_open, pond_server_poll, pond_server_query,
                   pond_server_stream_bytes, pond_server_submit, pond_server_take_profiles,
                   pond_stream_desc, pond_completion, _desc as stream_desc, pond_aid_create,
                   pond_aid_destroy, pond_aid_geometry, pond_aid_run, POND_LSB, POND_USB, SIDEBANDS,
                   POND_INPUT_COMPLEX, POND_INPUT_REAL_LSB, POND_INPUT_REAL_USB, pond_real_plan_create,
                   pond_real_dedisperse, pond_real_expect, pond_copy_device, pond_geometry,
                   pond_server_stream_state, POND_ECANCELED, POND_TICKET_ADMITTED, POND_STREAM_WAITING,
                   POND_STREAM_OPEN, POND_STREAM_CLOSED, pond_dedisperse_segment_noalloc,
                   POND_BATCH_AUTOTUNE, pond_plan_autotune, pond_search_autotune, POND_BF16)
