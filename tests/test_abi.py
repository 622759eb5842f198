"""The C ABI without a GPU: libnrm.so loads, exports every function that
include/nrm.h declares, and rejects bad arguments on the host before any HIP
call is made (no compute is launched here)."""
import ctypes
import os
import re

import pytest

from paper_2207_00257_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s*([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                             text, flags=re.M):
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2207_00257_amd import build

        build.build()
    return L.lib()


def test_header_declares_the_north_star_calls():
    names = declared_functions()
    assert "normalize" in names and "nrm_normalize_ex" in names, names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_status_strings(lib):
    for st in (L.NRM_OK, L.NRM_EINVAL, L.NRM_EOVERLAP, L.NRM_ENOMEM, L.NRM_EHIP, L.NRM_EUNSUPPORTED,
               L.NRM_EDEVICE):
        assert lib.nrm_status_string(st)
    assert lib.nrm_status_string(12345) == b"unknown status"


def test_host_validation_before_any_hip_call(lib):
    ex = lib.nrm_normalize_ex
    assert ex(None, 0, 0, 0, 0, -1, 0, None) == L.NRM_EINVAL           # n < 0
    assert ex(None, 0, 0, 0, 0, 0, 0, None) == L.NRM_OK                # n == 0: no-op
    assert ex(None, 0, 0, 4096, 0, 10, 0, None) == L.NRM_EINVAL        # NULL out
    assert ex(None, 4096, 0, 0, 0, 10, 0, None) == L.NRM_EINVAL        # NULL in
    assert ex(None, 4096, 7, 8192, 0, 10, 0, None) == L.NRM_EINVAL     # bad out dtype
    assert ex(None, 4096, 0, 8192, 9, 10, 0, None) == L.NRM_EINVAL     # bad in dtype
    assert ex(None, 4096, 0, 8192, 0, 10, 5, None) == L.NRM_EINVAL     # bad accumulation
    assert ex(None, 4100, 0, 4096, 0, 10, 0, None) == L.NRM_EOVERLAP   # out starts inside in
    assert ex(None, 4096, 0, 4100, 0, 10, 0, None) == L.NRM_EOVERLAP   # in starts inside out
    assert ex(None, 4096, 0, 4096, 1, 10, 0, None) == L.NRM_EOVERLAP   # same base, f32 out over bf16 in
    assert lib.normalize(None, None, -5) == L.NRM_EINVAL
    assert lib.normalize(None, None, 0) == L.NRM_OK
    assert lib.nrm_set_params(None, None) == L.NRM_EINVAL
    assert lib.nrm_create(None, 0) == L.NRM_EINVAL
    assert lib.nrm_destroy(None) == L.NRM_OK
