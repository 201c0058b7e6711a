"""ctypes loader for libqai.so (the C ABI declared in include/qai.h).

torch is imported first so that the library binds to the HIP runtime torch
already loaded (one runtime per process).  There is no fallback: if the
library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library then shares)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqai.so")

QAI_OK = 0
QAI_BATCH_AUTOTUNE = 0x1
QAI_BATCH_TUNE_EACH = 0x2
BLOCK_MODES = {"ep": 0, "approximate": 1}
ERRORS = {-1: "QAI_EINVAL", -2: "QAI_EDIMS", -3: "QAI_ENOWS", -4: "QAI_EHIP", -5: "QAI_ENODEV",
          -6: "QAI_ESTATE"}
QAI_STATUS_QRANGE = 0x1
MAX_EXTENT = 16384
NOALLOC_SCRATCH_BYTES = 256 << 20


class QAIError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_float), ("power", ctypes.c_float), ("flags", ctypes.c_uint32)]


class Taps(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("q", "b1", "sb", "s", "d1sq", "b2", "d2sq", "w")]


class Tuning(ctypes.Structure):
    _fields_ = [("edt1_algo", ctypes.c_int32 * 2), ("edt2_algo", ctypes.c_int32 * 2), ("edt1_ring", ctypes.c_int32),
                ("edt2_ring", ctypes.c_int32), ("tile_log2", ctypes.c_int32 * 2), ("seed_rows", ctypes.c_int32),
                ("seed_planes", ctypes.c_int32), ("window_threads", ctypes.c_int32), ("force_wide", ctypes.c_int32)]


class Coded(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("meta", ctypes.c_void_p), ("payload", ctypes.c_void_p),
                ("payload_words", ctypes.c_uint64), ("seg_len", ctypes.c_int32)]


Dims = ctypes.c_int64 * 3

EXPORTS = ["qai_mitigate", "qai_workspace_bytes", "qai_mitigate_ex", "qai_backward", "qai_device_status",
           "qai_last_error", "qai_batch_workspace_bytes", "qai_batch_plan_create", "qai_batch_plan_launch",
           "qai_batch_plan_launch_per_field", "qai_batch_plan_tuning", "qai_batch_plan_destroy", "qai_copy_probe",
           "qai_profile_enable", "qai_stage_times", "qai_tuning_get", "qai_tuning_set", "qai_mitigate_noalloc",
           "qai_autotune", "qai_tuning_cache_save", "qai_tuning_cache_load", "qai_tuning_cache_clear",
           "qai_tuning_cache_size", "qai_quality_workspace_bytes", "qai_quality", "qai_blocks_workspace_bytes",
           "qai_mitigate_blocks", "qai_decode", "qai_mitigate_coded"]

_lib = None


def load(path=LIB_PATH):
    """Load (once) and type the library; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libqai.so not built at {path}: run __graft_entry__.build() "
                          "or python -m paper_2602_20097_amd.build")
    lib = ctypes.CDLL(path)
    P, I64P, F, SZ, I = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_float, ctypes.c_size_t, ctypes.c_int
    lib.qai_mitigate.argtypes = [P, I64P, F, P, P]
    lib.qai_mitigate_noalloc.argtypes = [P, I64P, F, ctypes.POINTER(Params), P, P]
    lib.qai_workspace_bytes.argtypes = [I64P]
    lib.qai_workspace_bytes.restype = SZ
    lib.qai_mitigate_ex.argtypes = [P, I64P, F, ctypes.POINTER(Params), P, SZ, P, ctypes.POINTER(Taps), P]
    lib.qai_backward.argtypes = [P, P, SZ, I64P, F, ctypes.POINTER(Params), P, P]
    lib.qai_device_status.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint32)]
    lib.qai_last_error.restype = ctypes.c_char_p
    lib.qai_last_error.argtypes = []
    lib.qai_batch_workspace_bytes.argtypes = [I, ctypes.POINTER(Dims)]
    lib.qai_batch_workspace_bytes.restype = SZ
    lib.qai_batch_plan_create.argtypes = [I, ctypes.POINTER(P), ctypes.POINTER(Dims), ctypes.POINTER(F),
                                          ctypes.POINTER(P), ctypes.POINTER(Params), ctypes.c_uint32, P, SZ, P,
                                          ctypes.POINTER(P)]
    lib.qai_batch_plan_tuning.argtypes = [P, I, ctypes.POINTER(Tuning)]
    lib.qai_batch_plan_launch.argtypes = [P, P]
    lib.qai_batch_plan_launch_per_field.argtypes = [P, P]
    lib.qai_batch_plan_destroy.argtypes = [P]
    lib.qai_batch_plan_destroy.restype = None
    lib.qai_copy_probe.argtypes = [P, P, SZ, P]
    lib.qai_profile_enable.argtypes = [I]
    lib.qai_tuning_get.argtypes = [ctypes.POINTER(Tuning)]
    lib.qai_tuning_set.argtypes = [ctypes.POINTER(Tuning)]
    lib.qai_autotune.argtypes = [P, I64P, F, P, SZ, P, P, ctypes.POINTER(Tuning)]
    lib.qai_tuning_cache_save.argtypes = [ctypes.c_char_p]
    lib.qai_tuning_cache_load.argtypes = [ctypes.c_char_p]
    lib.qai_tuning_cache_clear.argtypes = []
    lib.qai_tuning_cache_size.argtypes = []
    lib.qai_quality_workspace_bytes.argtypes = [I64P]
    lib.qai_quality_workspace_bytes.restype = SZ
    lib.qai_quality.argtypes = [P, P, I64P, P, SZ, P, P]
    I32P = ctypes.POINTER(ctypes.c_int32)
    lib.qai_blocks_workspace_bytes.argtypes = [I64P, I32P, I]
    lib.qai_blocks_workspace_bytes.restype = SZ
    lib.qai_mitigate_blocks.argtypes = [P, I64P, F, ctypes.POINTER(Params), I32P, I, P, SZ, P, P]
    lib.qai_decode.argtypes = [ctypes.POINTER(Coded), I64P, F, P, P]
    lib.qai_mitigate_coded.argtypes = [ctypes.POINTER(Coded), I64P, F, ctypes.POINTER(Params), P, SZ, P, P]
    lib.qai_stage_times.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_char_p), I,
                                    ctypes.POINTER(I), I]
    for name in EXPORTS:
        if name not in ("qai_workspace_bytes", "qai_last_error", "qai_batch_workspace_bytes",
                        "qai_batch_plan_destroy", "qai_quality_workspace_bytes", "qai_blocks_workspace_bytes"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc):
    if rc != QAI_OK:
        msg = _lib.qai_last_error().decode(errors="replace") if _lib is not None else ""
        raise QAIError(rc, msg)
    return rc


def dims3(shape):
    shape = tuple(int(s) for s in shape)
    if not 1 <= len(shape) <= 3:
        raise ValueError(f"field must be 1-, 2- or 3-D, got shape {shape}")
    shape = (1,) * (3 - len(shape)) + shape
    return Dims(*shape)
