"""CPU oracle for the QAI post-pass -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It wraps ``qai_oracle.c`` (plain FP64 C following
Algorithms 1-4 of the paper) through ctypes and shares nothing with the GPU
library.  See the header of ``qai_oracle.c`` for the readings it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qai_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")
INF = np.iinfo(np.int64).max

_lib = None


def build(force=True):
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", SRC, "-o", tmp, "-lm"]
    if force or not os.path.exists(LIB):
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    F = ctypes.c_float
    lib.orc_qai.argtypes = [P, I64, I64, I64, F, F, F, P, P, P, P, P, P, P, P, P, P]
    lib.orc_qai.restype = ctypes.c_int
    lib.orc_edt.argtypes = [P, I64, I64, I64, P, P]
    lib.orc_edt.restype = ctypes.c_int
    lib.orc_recover_q.argtypes = [P, I64, F, P]
    lib.orc_recover_q.restype = ctypes.c_int
    lib.orc_boundary_sign.argtypes = [P, I64, I64, I64, P, P]
    lib.orc_boundary_sign.restype = None
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dims(shape):
    shape = tuple(int(s) for s in shape)
    while len(shape) < 3:
        shape = (1,) + shape
    return shape


def max_threads():
    return int(_load().orc_max_threads())


def qai(xq, eb, eta=0.9, power=1.0):
    """Run Algorithm 4 on a decompressed float32 field.

    Returns a dict with ``out`` (float64) and every intermediate: ``q``
    (int32), ``b1`` (uint8), ``sb`` (int8, boundary sign), ``d1sq`` (int64,
    -1 where no boundary exists), ``i1`` (int64 linear index of the nearest
    boundary, -1 if none), ``s`` (int8 propagated sign), ``b2`` (uint8),
    ``d2sq`` (int64, -1 if none) and ``w`` (float64 interpolation weight).
    """
    lib = _load()
    xq = np.ascontiguousarray(xq, dtype=np.float32)
    nz, ny, nx = _dims(xq.shape)
    n = xq.size
    r = dict(out=np.empty(n, np.float64), q=np.empty(n, np.int32), b1=np.empty(n, np.uint8),
             sb=np.empty(n, np.int8), d1sq=np.empty(n, np.int64), i1=np.empty(n, np.int64),
             s=np.empty(n, np.int8), b2=np.empty(n, np.uint8), d2sq=np.empty(n, np.int64),
             w=np.empty(n, np.float64))
    rc = lib.orc_qai(_ptr(xq), nz, ny, nx, float(np.float32(eb)), float(np.float32(eta)),
                     float(np.float32(power)), _ptr(r["out"]), _ptr(r["q"]), _ptr(r["b1"]),
                     _ptr(r["sb"]), _ptr(r["d1sq"]), _ptr(r["i1"]), _ptr(r["s"]), _ptr(r["b2"]),
                     _ptr(r["d2sq"]), _ptr(r["w"]))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    for k in ("d1sq", "d2sq"):
        r[k][r[k] == INF] = -1
    for k in r:
        r[k] = r[k].reshape(xq.shape)
    return r


def edt(mask):
    """Squared EDT to the nonzero voxels of ``mask`` (Algorithm 1 per axis)
    and the feature transform (nearest seed's linear index).  -1 = none."""
    lib = _load()
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = _dims(m.shape)
    d = np.empty(m.size, np.int64)
    f = np.empty(m.size, np.int64)
    rc = lib.orc_edt(_ptr(m), nz, ny, nx, _ptr(d), _ptr(f))
    if rc != 0:
        raise MemoryError("oracle EDT failed")
    d[d == INF] = -1
    return d.reshape(m.shape), f.reshape(m.shape)


def boundary_sign(q):
    """Algorithm 2 on an int32 index field: returns (B1, S_B)."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.int32)
    nz, ny, nx = _dims(q.shape)
    b = np.empty(q.size, np.uint8)
    s = np.empty(q.size, np.int8)
    lib.orc_boundary_sign(_ptr(q), nz, ny, nx, _ptr(b), _ptr(s))
    return b.reshape(q.shape), s.reshape(q.shape)


def recover_q(xq, eb):
    lib = _load()
    xq = np.ascontiguousarray(xq, dtype=np.float32)
    q = np.empty(xq.size, np.int32)
    rc = lib.orc_recover_q(_ptr(xq), xq.size, float(np.float32(eb)), _ptr(q))
    if rc != 0:
        raise ValueError("index out of range")
    return q.reshape(xq.shape)
