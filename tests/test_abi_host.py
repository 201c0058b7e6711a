"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/qai.h declares, sizes workspaces, and rejects bad arguments on the
host before anything is enqueued."""
import ctypes
import math
import os
import re

import pytest

from paper_2602_20097_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qai.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qai_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "qai_mitigate" in names and "qai_mitigate_ex" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_workspace_bytes(lib):
    for shape in ((1, 1, 1), (64, 64, 64), (256, 384, 384), (1, 1800, 3600), (3, 5, 7)):
        n = math.prod(shape)
        b = lib.qai_workspace_bytes(_lib.Dims(*shape))
        cap = shape[0] * ((shape[1] + 3) // 4) * 4 * shape[2]
        words = 3 * (((cap * 4) + 255) // 256) * 256
        bits = (((n + 1023) // 1024 * 128 + 255) // 256) * 256
        assert b == 64 * 1024 + words + bits
    for bad in ((0, 4, 4), (4, -1, 4), (1, 1, 16385)):
        assert lib.qai_workspace_bytes(_lib.Dims(*bad)) == 0
    assert lib.qai_workspace_bytes(None) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def call_ex(lib, field=FAKE, dims=(4, 4, 4), eb=0.1, params=None, ws=FAKE, ws_bytes=1 << 30, out=FAKE):
    prm = ctypes.byref(params) if params is not None else None
    d = _lib.Dims(*dims) if dims is not None else None
    return lib.qai_mitigate_ex(field, d, ctypes.c_float(eb), prm, ws, ws_bytes, out, None, None)


def test_argument_errors_are_caught_on_the_host(lib):
    assert call_ex(lib, dims=(0, 4, 4)) == -2
    assert call_ex(lib, dims=(4, 4, 20000)) == -2
    assert call_ex(lib, dims=None) == -1
    assert call_ex(lib, field=None) == -1
    assert call_ex(lib, out=None) == -1
    for eb in (0.0, -1.0, float("nan"), float("inf"), 1e-45):
        assert call_ex(lib, eb=eb) == -1, eb
    assert call_ex(lib, params=_lib.Params(float("nan"), 1.0, 0)) == -1
    assert call_ex(lib, params=_lib.Params(0.9, 0.0, 0)) == -1
    assert call_ex(lib, params=_lib.Params(0.9, 1.0, 1)) == -1
    assert call_ex(lib, ws=None) == -3
    assert call_ex(lib, ws_bytes=100) == -3
    assert call_ex(lib, ws=ctypes.c_void_p(0x1010)) == -3  # misaligned
    # out overlapping field partly
    assert call_ex(lib, field=ctypes.c_void_p(0x100000), out=ctypes.c_void_p(0x100004)) == -1
    msg = lib.qai_last_error().decode()
    assert "overlap" in msg
    assert lib.qai_mitigate(FAKE, _lib.Dims(4, 0, 4), ctypes.c_float(0.1), FAKE, None) == -2
    assert lib.qai_backward(None, FAKE, 1 << 30, _lib.Dims(4, 4, 4), ctypes.c_float(0.1), None, FAKE, None) == -1
    assert lib.qai_copy_probe(None, FAKE, 4, None) == -1
    # the allocation-free entry point: size limit of its fixed scratch, bad dims
    big = _lib.Dims(512, 512, 512)
    assert lib.qai_workspace_bytes(big) > _lib.NOALLOC_SCRATCH_BYTES
    assert lib.qai_mitigate_noalloc(FAKE, big, ctypes.c_float(0.1), None, FAKE, None) == -3
    assert "scratch" in lib.qai_last_error().decode()
    assert lib.qai_mitigate_noalloc(FAKE, _lib.Dims(4, 0, 4), ctypes.c_float(0.1), None, FAKE, None) == -2


def test_no_device_is_reported_without_a_launch(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present; this checks the no-device path")
    except Exception:
        pass
    assert call_ex(lib) == -5
    assert "GPU" in lib.qai_last_error().decode()


def test_batch_workspace_and_argument_errors(lib):
    dims = (_lib.Dims * 3)(_lib.Dims(4, 5, 6), _lib.Dims(1, 1, 1000), _lib.Dims(2, 300, 7))
    want = sum(((lib.qai_workspace_bytes(dims[i]) + 255) // 256) * 256 for i in range(3))
    assert lib.qai_batch_workspace_bytes(3, dims) == want
    assert lib.qai_batch_workspace_bytes(0, dims) == 0
    bad = (_lib.Dims * 1)(_lib.Dims(4, 0, 6))
    assert lib.qai_batch_workspace_bytes(1, bad) == 0
    P = ctypes.c_void_p
    fp = (P * 1)(0x1000)
    op = (P * 1)(0x100000)
    eb = (ctypes.c_float * 1)(0.5)
    d1 = (_lib.Dims * 1)(_lib.Dims(4, 5, 6))
    h = ctypes.c_void_p()
    big = 1 << 30
    assert lib.qai_batch_plan_create(0, fp, d1, eb, op, None, 0, FAKE, big, None, ctypes.byref(h)) == -1
    assert lib.qai_batch_plan_create(1, fp, d1, eb, op, None, 4, FAKE, big, None, ctypes.byref(h)) == -1
    assert lib.qai_batch_plan_create(1, fp, bad, eb, op, None, 0, FAKE, big, None, ctypes.byref(h)) == -2
    ebz = (ctypes.c_float * 1)(0.0)
    assert lib.qai_batch_plan_create(1, fp, d1, ebz, op, None, 0, FAKE, big, None, ctypes.byref(h)) == -1
    same = (P * 1)(0x1000)
    assert lib.qai_batch_plan_create(1, fp, d1, eb, same, None, 0, FAKE, big, None, ctypes.byref(h)) == -1
    assert lib.qai_batch_plan_create(1, fp, d1, eb, op, None, 0, None, big, None, ctypes.byref(h)) == -3
    assert lib.qai_batch_plan_create(1, fp, d1, eb, op, None, 0, FAKE, 10, None, ctypes.byref(h)) == -3
    assert h.value is None
    assert lib.qai_batch_plan_launch(None, None) == -6
    assert lib.qai_batch_plan_tuning(None, 0, None) == -1


def test_tuning_cache_file_round_trip(lib, tmp_path):
    """The per-shape tuning cache is host state: load validates every line,
    save writes back what was loaded, a malformed file adds nothing."""
    assert lib.qai_tuning_cache_clear() == 0
    assert lib.qai_tuning_cache_size() == 0
    good = tmp_path / "cache.txt"
    rows = ["1 1800 3600 -1 1 -1 1 16 32 5 4 0 16 512", "100 500 500 4 4 3 3 16 32 -1 -1 0 32 256"]
    good.write_text("qai-tuning-cache 1\n" + "\n".join(rows) + "\n")
    assert lib.qai_tuning_cache_load(str(good).encode()) == 0
    assert lib.qai_tuning_cache_size() == 2
    out = tmp_path / "saved.txt"
    assert lib.qai_tuning_cache_save(str(out).encode()) == 0
    lines = out.read_text().splitlines()
    assert lines[0] == "qai-tuning-cache 1"
    assert sorted(lines[1:]) == sorted(rows)
    for bad_row in ("1 1800 3600 -1 1 -1 1 16 33 5 4 0 16 512",   # ring size
                    "1 1800 3600 -1 1 -1 1 16 32 5 4 0 16 500",   # workgroup size
                    "0 1800 3600 -1 1 -1 1 16 32 5 4 0 16 512",   # extent
                    "1 1800 3600 -1 1 -1"):                       # short line
        bad = tmp_path / "bad.txt"
        bad.write_text("qai-tuning-cache 1\n64 64 64 -1 -1 -1 -1 16 32 -1 -1 0 16 256\n" + bad_row + "\n")
        assert lib.qai_tuning_cache_load(str(bad).encode()) == -1, bad_row
        assert lib.qai_tuning_cache_size() == 2
    nohdr = tmp_path / "nohdr.txt"
    nohdr.write_text(rows[0] + "\n")
    assert lib.qai_tuning_cache_load(str(nohdr).encode()) == -1
    assert lib.qai_tuning_cache_load(str(tmp_path / "missing.txt").encode()) == -1
    assert lib.qai_tuning_cache_clear() == 0
    assert lib.qai_tuning_cache_size() == 0


def test_coded_argument_errors(lib):
    base = ctypes.c_void_p(0x1000)
    c = _lib.Coded(0x1000, 0x2000, 0x3000, 10, 32)
    d = _lib.Dims(4, 4, 40)
    assert lib.qai_mitigate_coded(None, d, ctypes.c_float(0.1), None, FAKE, 1 << 30, FAKE, None) == -1
    bad = _lib.Coded(0x1000, 0x2000, 0x3000, 10, 16)
    assert lib.qai_mitigate_coded(ctypes.byref(bad), d, ctypes.c_float(0.1), None, FAKE, 1 << 30, FAKE, None) == -1
    assert "32" in lib.qai_last_error().decode()
    empty = _lib.Coded(0x1000, 0x2000, 0x3000, 0, 32)
    assert lib.qai_decode(ctypes.byref(empty), d, ctypes.c_float(0.1), FAKE, None) == -1
    assert lib.qai_decode(ctypes.byref(c), _lib.Dims(0, 4, 4), ctypes.c_float(0.1), FAKE, None) == -2
    assert lib.qai_mitigate_coded(ctypes.byref(c), d, ctypes.c_float(0.1), None, FAKE, 10, FAKE, None) == -3
    del base
