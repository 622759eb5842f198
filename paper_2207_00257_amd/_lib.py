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
NRM_LAYOUT_CHUNK, NRM_LAYOUT_STRIDE = 0, 1


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
        ("reserved", ctypes.c_int32 * 4),
    ]


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
        "nrm_status_string": (ctypes.c_char_p, [i32]),
        "nrm_last_error": (ctypes.c_char_p, []),
        "nrm_set_timing": (i32, [p, i32]),
        "nrm_kernel_times": (i32, [p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]),
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
