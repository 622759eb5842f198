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


def test_header_declares_the_basic_calls():
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


def test_batched_host_validation_before_any_hip_call(lib):
    ex = lib.nrm_normalize_batched_ex
    offs = 1 << 20  # an address only used for its non-NULL value; nothing is read at it
    assert ex(None, 4096, 0, 8192, 0, offs, -1, 10, 0, None) == L.NRM_EINVAL   # rows < 0
    assert ex(None, 4096, 0, 8192, 0, offs, 0, 10, 0, None) == L.NRM_OK        # no rows
    assert ex(None, 4096, 0, 8192, 0, None, 3, 10, 0, None) == L.NRM_EINVAL    # NULL offsets
    assert ex(None, 4096, 0, 8192, 0, offs, 3, 0, 0, None) == L.NRM_OK         # zero capacity
    assert ex(None, 4096, 5, 8192, 0, offs, 3, 10, 0, None) == L.NRM_EINVAL    # bad dtype
    assert ex(None, 4096, 0, 8192, 0, offs, 3, 10, 7, None) == L.NRM_EINVAL    # bad accumulation
    assert ex(None, None, 0, 8192, 0, offs, 3, 10, 0, None) == L.NRM_EINVAL    # NULL out
    assert ex(None, 4097, 0, 8192, 0, offs, 3, 10, 0, None) == L.NRM_EINVAL    # misaligned out
    assert ex(None, 4100, 0, 4096, 0, offs, 3, 10, 0, None) == L.NRM_EOVERLAP  # partial overlap
    sm = lib.nrm_softmax_batched
    assert sm(None, 4096, 8192, offs, -1, 10, None, None) == L.NRM_EINVAL    # rows < 0
    assert sm(None, 4096, 8192, offs, 0, 10, None, None) == L.NRM_OK         # no rows
    assert sm(None, 4096, 8192, None, 3, 10, None, None) == L.NRM_EINVAL     # NULL offsets
    assert sm(None, 4096, 8192, offs, 3, 0, None, None) == L.NRM_OK          # zero capacity, no lse
    assert sm(None, 4096, 8192, offs, 3, 10, 65538, None) == L.NRM_EINVAL    # misaligned lse
    assert sm(None, None, 8192, offs, 3, 10, None, None) == L.NRM_EINVAL     # NULL out
    assert sm(None, 4100, 4096, offs, 3, 10, None, None) == L.NRM_EOVERLAP   # in and out partly overlap
    assert sm(None, 4096, 8192, offs, 3, 10, 8200, None) == L.NRM_EOVERLAP   # lse inside in
    assert sm(None, 4096, 8192, offs, 3, 10, 4092, None) == L.NRM_EOVERLAP   # lse runs into out
    rows = (L.NrmRow * 2)()
    rows[0].in_, rows[0].out, rows[0].n = 8192, 4096, 4
    rows[1].in_, rows[1].out, rows[1].n = 16384, 12288, -1
    nr = lib.nrm_normalize_rows
    assert nr(None, rows, -1, 0, None) == L.NRM_EINVAL
    assert nr(None, rows, 0, 0, None) == L.NRM_OK
    assert nr(None, None, 2, 0, None) == L.NRM_EINVAL
    assert nr(None, rows, 2, 0, None) == L.NRM_EINVAL          # n < 0
    rows[1].n, rows[1].in_dtype = 4, 9
    assert nr(None, rows, 2, 0, None) == L.NRM_EINVAL          # bad dtype
    rows[1].in_dtype, rows[1].out = 0, 16388
    assert nr(None, rows, 2, 0, None) == L.NRM_EOVERLAP        # row overlaps itself
    rows[1].out = 12288
    assert nr(None, rows, 2, 5, None) == L.NRM_EINVAL          # bad accumulation
    p = L.NrmBatchParams()
    assert lib.nrm_default_batch_params(ctypes.byref(p)) == L.NRM_OK
    assert p.block >= 64 and p.tile_log2 >= 10
    assert lib.nrm_set_batch_params(None, ctypes.byref(p)) == L.NRM_EINVAL
    assert lib.nrm_batch_reserve(None, 1, 1) == L.NRM_EINVAL


def test_nll_validation_before_any_hip_call(lib):
    f = lib.nrm_nll_loss
    lp, tg, w = 1 << 20, 1 << 22, 1 << 24  # addresses used only for their values; nothing is read
    assert f(None, 4096, None, lp, tg, w, -1, 10, -100, 2, 0, None) == L.NRM_EINVAL      # n < 0
    assert f(None, 4096, None, lp, tg, w, 5, 0, -100, 2, 0, None) == L.NRM_EINVAL        # no classes
    assert f(None, 4096, None, lp, tg, w, 5, 10, -100, 3, 0, None) == L.NRM_EINVAL       # reduction
    assert f(None, 4096, None, lp, tg, w, 5, 10, -100, 2, 9, None) == L.NRM_EINVAL       # accumulation
    assert f(None, 4096, None, lp, tg, w, 0, 10, -100, 0, 0, None) == L.NRM_OK           # none of nothing
    assert f(None, None, None, lp, tg, w, 5, 10, -100, 2, 0, None) == L.NRM_EINVAL       # NULL out
    assert f(None, 4096, None, None, tg, w, 5, 10, -100, 2, 0, None) == L.NRM_EINVAL     # NULL logp
    assert f(None, 4096, None, lp, tg + 4, w, 5, 10, -100, 2, 0, None) == L.NRM_EINVAL   # misaligned target
    assert f(None, lp + 8, None, lp, tg, w, 5, 10, -100, 2, 0, None) == L.NRM_EOVERLAP   # out inside logp
    assert f(None, 4096, tg, lp, tg, w, 5, 10, -100, 2, 0, None) == L.NRM_EOVERLAP       # total weight on target
    assert f(None, 4096, 4096, lp, tg, w, 5, 10, -100, 2, 0, None) == L.NRM_EOVERLAP     # out on total weight
    assert f(None, 4096, None, lp, tg, w, 1 << 40, 1 << 40, -100, 2, 0, None) == L.NRM_EINVAL  # N * C too large


def test_layerforward_validation_before_any_hip_call(lib):
    f = lib.nrm_layerforward
    h, i, o = 1 << 20, 1 << 24, 1 << 26
    assert f(4, h, i, o, 16, None) == L.NRM_EINVAL            # unknown form
    assert f(0, h, i, o, 17, None) == L.NRM_EINVAL            # not whole tiles
    assert f(0, h, i, o, -16, None) == L.NRM_EINVAL
    assert f(0, h, i, o, 0, None) == L.NRM_OK                 # nothing to do
    assert f(0, None, i, o, 16, None) == L.NRM_EINVAL
    assert f(0, h + 2, i, o, 16, None) == L.NRM_EINVAL        # misaligned
    assert f(0, h, h + 64, o, 16, None) == L.NRM_EOVERLAP     # input inside hidden
    assert f(1, h, i, i + 32, 16, None) == L.NRM_EOVERLAP     # output overlaps input


def test_server_config_validation_before_any_hip_call(lib):
    cfg = L.NrmServerConfig()
    assert lib.nrm_server_default_config(ctypes.byref(cfg)) == L.NRM_OK
    assert cfg.slots >= 1 and cfg.budget_bytes == 64 << 30 and cfg.batching == 1
    assert cfg.spread == 1 and cfg.single_plain == 1
    h = ctypes.c_void_p()
    for field, bad in (("slots", 0), ("slots", 65), ("budget_bytes", 0), ("max_batch_rows", 0),
                       ("max_batch_elems", 0), ("batching", 2), ("graph", 5), ("accum", 3),
                       ("hold_outputs", 7), ("use_batch_params", 2), ("single_plain", 2), ("spread", -1),
                       ("idle_spin_us", -1), ("idle_spin_us", 1000001), ("min_batch_rows", 0),
                       ("device_queue", 2)):
        c = L.NrmServerConfig()
        lib.nrm_server_default_config(ctypes.byref(c))
        setattr(c, field, bad)
        assert lib.nrm_server_create(ctypes.byref(h), 0, ctypes.byref(c)) == L.NRM_EINVAL, field
    # the device queue's own limits (checked with device_queue = 1)
    assert cfg.device_queue == 0 and cfg.dq_blocks == 0 and cfg.dq_idle_us == 100000
    assert cfg.dq_plain_above == 1 << 20 and cfg.dq_slice_us == 10000
    for field, bad in (("dq_blocks", 63), ("dq_blocks", (1 << 16) + 1), ("dq_idle_us", 0),
                       ("dq_idle_us", 10000001), ("dq_plain_above", 0), ("dq_plain_above", (1 << 25) + 1),
                       ("dq_slice_us", -1), ("dq_slice_us", 10000001)):
        c = L.NrmServerConfig()
        lib.nrm_server_default_config(ctypes.byref(c))
        c.device_queue = 1
        setattr(c, field, bad)
        assert lib.nrm_server_create(ctypes.byref(h), 0, ctypes.byref(c)) == L.NRM_EINVAL, field
    assert lib.nrm_server_create(None, 0, ctypes.byref(cfg)) == L.NRM_EINVAL
    assert lib.nrm_server_submit(None, None, 0) == L.NRM_EINVAL
    assert lib.nrm_server_destroy(None) == L.NRM_OK


def test_forms_validation_before_any_hip_call(lib):
    f = lib.nrm_normalize_form
    assert f(0, 4096, 8192, 10, 256, None) == L.NRM_EINVAL          # unknown form
    assert f(1, 4096, 8192, 0, 256, None) == L.NRM_EINVAL           # n < 1
    assert f(1, 4096, 8192, (1 << 20) + 1, 256, None) == L.NRM_EINVAL
    assert f(2, 4096, 8192, 10, 100, None) == L.NRM_EINVAL          # block not a multiple of 64
    assert f(2, None, 8192, 10, 256, None) == L.NRM_EINVAL
    assert f(1, 4098, 8192, 10, 256, None) == L.NRM_EINVAL          # misaligned
    assert f(1, 4096, 4096, 10, 256, None) == L.NRM_EOVERLAP        # in place is not allowed here


def test_height_cap_keeps_the_stated_bound():
    """nrm_params.max_height is capped so that the worst case the header
    states, gamma_h + u with h = max_height + 26 and u = 2^-24, stays within
    the 4e-6 relative tolerance: 40 is the largest cap for which it does."""
    text = open(os.path.join(ROOT, "include", "nrm.h")).read()
    m = re.search(r"int32_t max_height;.*?(\d+)\.\.(\d+)", text, flags=re.S)
    lo, hi = int(m.group(1)), int(m.group(2))
    u = 2.0 ** -24

    def bound(h):
        return h * u / (1 - h * u) + u

    assert lo == 24 and hi == 40
    assert bound(hi + 26) < 4e-6 < bound(hi + 27)
    src = open(os.path.join(ROOT, "paper_2207_00257_amd", "csrc", "nrm_api.cpp")).read()
    assert "p.max_height > %d" % hi in src


def test_tuning_cache_read_by_the_library(lib):
    """The library reads the committed tuning cache itself: the entry the
    autotuner stored for (gfx950, f32, f32, plain, 2^28), field by field; no
    entry for a size class it has not tuned; and a cache named by
    NRM_TUNE_CACHE (read once per process: checked in a child process)."""
    import json
    import subprocess
    import sys

    cache = json.load(open(os.path.join(ROOT, "paper_2207_00257_amd", "tuned", "plain.json")))
    want = cache["gfx950/f32->f32/f32/2^28"]["params"]
    p = L.NrmParams()
    assert lib.nrm_tuned_params(b"gfx950", 0, 0, 0, (1 << 28) + 5, ctypes.byref(p)) == 1
    for k, v in want.items():
        assert getattr(p, k) == v, k
    d = L.NrmParams()
    assert lib.nrm_default_params(ctypes.byref(d)) == L.NRM_OK
    assert lib.nrm_tuned_params(b"gfx950", 0, 0, 0, 1 << 12, ctypes.byref(p)) == 0
    assert bytes(p) == bytes(d)
    assert lib.nrm_tuned_params(b"gfx942", 0, 0, 0, 1 << 28, ctypes.byref(p)) == 0
    assert lib.nrm_tuned_params(None, 0, 0, 0, 1 << 28, ctypes.byref(p)) == L.NRM_EINVAL
    code = ("import ctypes, sys; sys.path.insert(0, %r); from paper_2207_00257_amd import _lib as L; "
            "p = L.NrmParams(); r = L.lib().nrm_tuned_params(b'gfxtest', 1, 0, 1, 3000, ctypes.byref(p)); "
            "print(r, p.block, p.map_grid, p.tile_log2)" % ROOT)
    import tempfile
    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
        json.dump({"gfxtest/bf16->f32/kahan/2^11": {"ms": 1.0, "params": {"block": 128, "map_grid": 77,
                                                                           "tile_log2": 11}},
                   "other": [1, 2, {"x": "y"}]}, f)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       env=dict(os.environ, NRM_TUNE_CACHE=f.name))
    os.unlink(f.name)
    assert r.stdout.split() == ["1", "128", "77", "11"], r.stdout + r.stderr


def _declared_prototypes():
    """name -> list of parameter types (text) from include/*.h."""
    protos = {}
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"#[^\n]*", "", text)
        for m in re.finditer(r"(?:^|;|\})\s*(?:const\s+)?[A-Za-z_]\w*\s*\**\s*([A-Za-z_]\w*)\s*\(([^;{)]*)\)\s*;",
                             text, flags=re.M):
            params = [p.strip() for p in m.group(2).replace("\n", " ").split(",") if p.strip()]
            if params == ["void"]:
                params = []
            protos[m.group(1)] = params
    return protos


def _kind_of_c(param):
    t = re.sub(r"\b[A-Za-z_]\w*$", "", param.strip()).strip()  # drop the parameter name
    t = t.replace("const ", "").strip()
    if "*" in t:
        return "char*" if t.replace(" ", "") == "char*" else "ptr"
    return {"int64_t": "i64", "int": "i32", "int32_t": "i32"}.get(t, t)


def _kind_of_ctypes(ct):
    if ct is ctypes.c_char_p:
        return "char*"
    if ct is ctypes.c_int64:
        return "i64"
    if ct is ctypes.c_int:
        return "i32"
    return "ptr"  # c_void_p and POINTER(...)


def test_binding_signatures_match_the_header(lib):
    """Every function the binding declares exists in include/nrm.h with the
    same number of parameters, each of the same kind (pointer, 32-bit or
    64-bit integer), so a marshalling slip cannot pass unnoticed."""
    protos = _declared_prototypes()
    checked = 0
    for name in dir(lib):
        fn = getattr(lib, name, None)
        args = getattr(fn, "argtypes", None)
        if name.startswith("_") or args is None:
            continue
        assert name in protos, name
        want = [_kind_of_c(p) for p in protos[name]]
        got = [_kind_of_ctypes(a) for a in args]
        assert want == got, (name, protos[name], got)
        checked += 1
    assert checked >= 35, checked  # every function the binding declares


def test_binding_struct_layouts_match_the_header(tmp_path):
    """Every public struct the Python binding declares has the size and field
    offsets that a C compiler gives it from include/nrm.h."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"nrm_params": L.NrmParams, "nrm_batch_params": L.NrmBatchParams, "nrm_row": L.NrmRow,
               "nrm_request": L.NrmRequest, "nrm_completion": L.NrmCompletion,
               "nrm_server_config": L.NrmServerConfig, "nrm_server_counters": L.NrmServerCounters}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "nrm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            cf = fname.rstrip("_")
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, cf))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", include, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
