"""ctypes loader for libnrm.so (the C ABI declared in include/nrm.h).

There is no fallback: if the library is not built, or the HIP runtime cannot
be loaded, importing the compute entry points raises. Build it with
`python -m paper_2207_00257_amd.build`.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnrm.so")

NRM_OK, NRM_EINVAL, NRM_EOVERLAP, NRM_ENOMEM, NRM_EHIP, NRM_EUNSUPPORTED, NRM_EDEVICE = (
    0, -1, -2, -3, -4, -5, -6)
NRM_F32, NRM_BF16, NRM_F16 = 0, 1, 2
NRM_ACC_F32, NRM_ACC_KAHAN = 0, 1
NRM_NLL_NONE, NRM_NLL_SUM, NRM_NLL_MEAN = 0, 1, 2
NRM_LAYOUT_CHUNK, NRM_LAYOUT_STRIDE = 0, 1
NRM_FORM_NAIVE, NRM_FORM_PERBLOCK = 1, 2
NRM_CEILING_COPY, NRM_CEILING_READ = 0, 1


class NrmParams(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("reduce_nt", ctypes.c_int32),
        ("max_height", ctypes.c_int32),
        ("map_block", ctypes.c_int32),
        ("map_unroll", ctypes.c_int32),
        ("map_grid", ctypes.c_int32),
        ("map_layout", ctypes.c_int32),
        ("map_nt", ctypes.c_int32),
        ("reverse_map", ctypes.c_int32),
        ("reduce_keep_mib", ctypes.c_int32),
        ("tile_log2", ctypes.c_int32),
        ("fused_combine", ctypes.c_int32),
        ("small_n", ctypes.c_int32),
        ("resident_n", ctypes.c_int32),
    ]


class NrmBatchParams(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("map_unroll", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("tile_log2", ctypes.c_int32),
        ("short_regs", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("map_block", ctypes.c_int32),
        ("map_grid", ctypes.c_int32),
        ("keep_mib", ctypes.c_int32),
        ("resident_segments", ctypes.c_int32),
        ("resident_grid", ctypes.c_int32),
        ("wave_max", ctypes.c_int32),
        ("wave_grid", ctypes.c_int32),
    ]


class NrmRow(ctypes.Structure):
    _fields_ = [
        ("in_", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("in_dtype", ctypes.c_int32),
        ("out_dtype", ctypes.c_int32),
    ]


class NrmRequest(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("in_", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("in_dtype", ctypes.c_int32),
        ("out_dtype", ctypes.c_int32),
        ("t_arrival_ns", ctypes.c_int64),
    ]


class NrmCompletion(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("out", ctypes.c_void_p),
        ("t_arrival_ns", ctypes.c_int64),
        ("t_launch_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class NrmServerConfig(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int32),
        ("batching", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("accum", ctypes.c_int32),
        ("hold_outputs", ctypes.c_int32),
        ("use_batch_params", ctypes.c_int32),
        ("single_plain", ctypes.c_int32),
        ("spread", ctypes.c_int32),
        ("idle_spin_us", ctypes.c_int32),
        ("min_batch_rows", ctypes.c_int32),
        ("budget_bytes", ctypes.c_int64),
        ("arena_bytes", ctypes.c_int64),
        ("max_batch_rows", ctypes.c_int64),
        ("max_batch_elems", ctypes.c_int64),
        ("batch_params", NrmBatchParams),
        ("device_queue", ctypes.c_int32),
        ("dq_blocks", ctypes.c_int32),
        ("dq_idle_us", ctypes.c_int64),
        ("dq_plain_above", ctypes.c_int64),
        ("dq_slice_us", ctypes.c_int64),
    ]


class NrmServerCounters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("in_flight", "queued", "held", "budget_used", "batches", "launches", "replaying", "failed")]


class NrmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s (status %d): %s" % (what, status, detail(status)))


_lib = None


def _declare(lib):
    i32, i64, p = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "normalize": (i32, [p, p, i64]),
        "nrm_create": (i32, [ctypes.POINTER(p), i32]),
        "nrm_destroy": (i32, [p]),
        "nrm_default_params": (i32, [ctypes.POINTER(NrmParams)]),
        "nrm_set_params": (i32, [p, ctypes.POINTER(NrmParams)]),
        "nrm_get_params": (i32, [p, ctypes.POINTER(NrmParams)]),
        "nrm_normalize_ex": (i32, [p, p, i32, p, i32, i64, i32, p]),
        "nrm_normalize_noalloc": (i32, [p, i32, p, i32, i64, i32, p]),
        "nrm_ceiling": (i32, [i32, p, p, i64, i64, p]),
        "nrm_tuned_params": (i32, [ctypes.c_char_p, i32, i32, i32, i64, ctypes.POINTER(NrmParams)]),
        "nrm_status_string": (ctypes.c_char_p, [i32]),
        "nrm_last_error": (ctypes.c_char_p, []),
        "nrm_set_timing": (i32, [p, i32]),
        "nrm_kernel_times": (i32, [p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]),
        "nrm_batch_times": (i32, [p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
        "normalize_batched": (i32, [p, p, p, i64]),
        "nrm_normalize_batched_ex": (i32, [p, p, i32, p, i32, p, i64, i64, i32, p]),
        "nrm_softmax_batched": (i32, [p, p, p, p, i64, i64, p, p]),
        "nrm_nll_loss": (i32, [p, p, p, p, p, p, i64, i64, i64, i32, i32, p]),
        "nrm_layerforward": (i32, [i32, p, p, p, i64, p]),
        "nrm_normalize_rows": (i32, [p, ctypes.POINTER(NrmRow), i64, i32, p]),
        "nrm_batch_reserve": (i32, [p, i64, i64]),
        "nrm_default_batch_params": (i32, [ctypes.POINTER(NrmBatchParams)]),
        "nrm_set_batch_params": (i32, [p, ctypes.POINTER(NrmBatchParams)]),
        "nrm_get_batch_params": (i32, [p, ctypes.POINTER(NrmBatchParams)]),
        "nrm_get_device_error": (i32, [p, p]),
        "nrm_get_last_sum": (i32, [p, p, ctypes.POINTER(ctypes.c_float)]),
        "nrm_normalize_form": (i32, [i32, p, p, i64, i32, p]),
        "nrm_server_default_config": (i32, [ctypes.POINTER(NrmServerConfig)]),
        "nrm_server_create": (i32, [ctypes.POINTER(p), i32, ctypes.POINTER(NrmServerConfig)]),
        "nrm_server_submit": (i32, [p, ctypes.POINTER(NrmRequest), i64]),
        "nrm_server_replay": (i32, [p, ctypes.POINTER(NrmRequest), i64, ctypes.POINTER(ctypes.c_int64)]),
        "nrm_server_poll": (i32, [p, ctypes.POINTER(NrmCompletion), i64, ctypes.POINTER(ctypes.c_int64)]),
        "nrm_server_release": (i32, [p, i64]),
        "nrm_server_last_failure": (i32, [p]),
        "nrm_server_stats": (i32, [p, ctypes.POINTER(NrmServerCounters)]),
        "nrm_server_destroy": (i32, [p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The loaded libnrm.so. Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnrm.so is not built (%s); run `python -m paper_2207_00257_amd.build`"
                               % LIB_PATH)
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def detail(status: int) -> str:
    L = lib()
    msg = L.nrm_status_string(status).decode()
    last = L.nrm_last_error().decode()
    return msg + (" - " + last if last else "")


def check(status: int, what: str) -> None:
    if status != NRM_OK:
        raise NrmError(status, what)
