"""ctypes front-end of the C FP64 oracle (oracle/csrc/oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  `build()` compiles
liboracle.so with gcc/OpenMP next to this file; `load()` returns the library,
building it when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csrc", "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DTYPE_CODE = {np.dtype(np.float32): 0, np.dtype(np.float16): 1, np.dtype(np.float64): 3}


def build():
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-ffp-contract=off", SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    i64, i32, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    lib.orc_philox.argtypes = [P, P, P]
    lib.orc_philox.restype = None
    lib.orc_hash.argtypes = [u64, i64, i32, i64, i64, P, P]
    lib.orc_hash.restype = ctypes.c_int
    lib.orc_sketch_f64.argtypes = [P, ctypes.c_int, i64, i64, i64, i64, i64, i32, u64,
                                   ctypes.c_double, P, ctypes.c_int]
    lib.orc_sketch_f64.restype = ctypes.c_int
    lib.orc_lstsq.argtypes = [P, ctypes.c_int, i64, i64, i64, P, P, ctypes.c_int]
    lib.orc_lstsq.restype = ctypes.c_int
    lib.orc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    load().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(v) for v in out)


def hash_rows(seed, row_begin, count, d, s):
    b = np.zeros((count, s), dtype=np.int64)
    g = np.zeros((count, s), dtype=np.int8)
    rc = load().orc_hash(seed, d, s, row_begin, count, _ptr(b), _ptr(g))
    if rc:
        raise ValueError("bad sketch shape")
    return b, g


def sketch_f64(A, d, s, seed, row_offset=0, scale=None, nthreads=0, bf16=False):
    """S[:, row_offset:+rows] @ A in FP64.  A: 2-D array (float32/float16/
    float64, or uint16 holding BF16 bits with bf16=True), row-major with any
    row stride (element units)."""
    A = np.asarray(A)
    if A.ndim != 2 or A.strides[1] != A.itemsize:
        A = np.ascontiguousarray(A)
    code = 2 if bf16 else DTYPE_CODE[A.dtype]
    rows, n = A.shape
    lda = A.strides[0] // A.itemsize
    if scale is None:
        scale = 1.0 / np.sqrt(float(s))
    SA = np.zeros((d, n), dtype=np.float64)
    rc = load().orc_sketch_f64(_ptr(A), code, rows, n, lda, row_offset, d, s, seed,
                               float(scale), _ptr(SA), int(nthreads))
    if rc:
        raise ValueError("orc_sketch_f64 failed: %d" % rc)
    return SA


def lstsq(A, b, nthreads=0):
    A = np.asarray(A)
    if A.strides[1] != A.itemsize:
        A = np.ascontiguousarray(A)
    m, n = A.shape
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n, dtype=np.float64)
    rc = load().orc_lstsq(_ptr(A), DTYPE_CODE[A.dtype], m, n, A.strides[0] // A.itemsize,
                          _ptr(b), _ptr(x), int(nthreads))
    if rc:
        raise ValueError("orc_lstsq failed: %d" % rc)
    return x


def max_threads():
    return int(load().orc_max_threads())
