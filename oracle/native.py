"""Build and load the oracle's plain C direct sum (test infrastructure).

`build()` compiles `direct_sum.c` with gcc into `_direct_sum.so` beside it.
`point_sum_c` calls it through ctypes.  gcc is used without fast-math, so
the C loop evaluates the same IEEE expressions as written.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct_sum.c")
_LIB = os.path.join(_HERE, "_direct_sum.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        f = lib.oracle_point_sum
        f.restype = None
        f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                      ctypes.c_void_p]
        _lib = lib
    return _lib


def point_sum_c(points, normals, weights, point_tri, k, a, b, rows=None):
    """Same contract as direct.point_sum, computed by the C loop."""
    lib = _load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    nrm = np.ascontiguousarray(normals, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    tri = np.ascontiguousarray(point_tri, dtype=np.int32)
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    batched = a.ndim == 3
    if not batched:
        a = a[None]
        b = b[None]
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    n = pts.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    y = np.zeros((a.shape[0], len(rows), 3), dtype=np.complex128)
    k = complex(k)
    lib.oracle_point_sum(n, pts.ctypes.data, nrm.ctypes.data, w.ctypes.data, tri.ctypes.data,
                         k.real, k.imag, a.shape[0], a.ctypes.data, b.ctypes.data,
                         len(rows), rows.ctypes.data, y.ctypes.data)
    return y if batched else y[0]
