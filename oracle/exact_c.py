"""ctypes wrapper of oracle/exact_maxtimes.c (test infrastructure only).

The exact (max, x) product of Alg. 2 (Sec. 2.2) for sizes where the numpy
formulation in ``pnorm.exact_maxtimes`` is too slow.  ``build_oracle_c``
compiles it with gcc; ``__graft_entry__.build()`` calls it, and the loader
calls it when the library is missing.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exact_maxtimes.c")
_LIB = os.path.join(_HERE, "liboracle_exact.so")
_lib = None


def build_oracle_c(force=True):
    """Compile exact_maxtimes.c into liboracle_exact.so (gcc, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_oracle_c(force=False)
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_exact_maxtimes_f64", "oracle_exact_maxtimes_f32in"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


def exact_maxtimes_c(A, B, rows=None):
    """R[t, j] = max_k A[rows[t], k] * B[k, j] in FP64 (all rows if rows is
    None).  A, B: 2-D FP32 or FP64 arrays."""
    lib = _load()
    if A.dtype == np.float32 and B.dtype == np.float32:
        fn = lib.oracle_exact_maxtimes_f32in
    else:
        A = np.asarray(A, dtype=np.float64)
        B = np.asarray(B, dtype=np.float64)
        fn = lib.oracle_exact_maxtimes_f64
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B)
    m_all, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    if rows is not None:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        if rows.size and (rows.min() < 0 or rows.max() >= m_all):
            raise IndexError("row index out of range")
        m = rows.size
        rp = rows.ctypes.data
    else:
        m = m_all
        rp = None
    R = np.empty((m, n), dtype=np.float64)
    fn(A.ctypes.data, B.ctypes.data, R.ctypes.data, m, k, n, rp)
    return R
