"""Python entry to the C certificate (oracle).  Test infrastructure only.

``certify(X, Y)`` returns the eq. (3) maximum over unordered pairs of the
eq. (2) distortion between rows of X (original points) and rows of Y (their
images), computed by direct differences in FP64 (``certificate.c``).
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "certificate.c")
_LIB = os.path.join(_HERE, "_certificate.so")
_lock = threading.Lock()
_lib = None


class OracleCert(ctypes.Structure):
    _fields_ = [("best", ctypes.c_double), ("second", ctypes.c_double),
                ("bi", ctypes.c_int64), ("bj", ctypes.c_int64),
                ("si", ctypes.c_int64), ("sj", ctypes.c_int64),
                ("bside", ctypes.c_int32), ("sside", ctypes.c_int32),
                ("nzero", ctypes.c_int64), ("npairs", ctypes.c_int64)]


def build(force=False):
    """Compile certificate.c with gcc -O2 -fopenmp into _certificate.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            i64, dp = ctypes.c_int64, ctypes.c_void_p
            lib.oracle_certificate.argtypes = [dp, dp, i64, i64, i64, i64, i64, ctypes.POINTER(OracleCert)]
            lib.oracle_certificate.restype = None
            lib.oracle_cross_certificate.argtypes = [dp, dp, i64, i64, dp, i64, dp, i64, ctypes.POINTER(OracleCert)]
            lib.oracle_cross_certificate.restype = None
            lib.oracle_pair_list.argtypes = [dp, dp, i64, i64, dp, dp, i64, dp, dp]
            lib.oracle_pair_list.restype = None
            lib.oracle_threads.argtypes = []
            lib.oracle_threads.restype = ctypes.c_int
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            lib.oracle_set_threads.restype = None
            _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def certify(X, Y, rows=None):
    """Max distortion over pairs (i < j).  ``rows=(i0, i1)`` restricts i to a
    block (all j > i still visited).  Returns a dict."""
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    if Y.ndim != 2 or Y.shape[0] != n:
        raise ValueError("Y must have one row per point")
    r = Y.shape[1]
    i0, i1 = (0, n) if rows is None else rows
    out = OracleCert()
    _load().oracle_certificate(X.ctypes.data, Y.ctypes.data, n, d, r, i0, i1, ctypes.byref(out))
    return {"max": out.best, "i": out.bi, "j": out.bj, "side": out.bside,
            "runner_up": out.second, "i2": out.si, "j2": out.sj, "side2": out.sside,
            "n_zero": out.nzero, "n_pairs": out.npairs}


def certify_cross(X, Y, IA, IB):
    """Max distortion over the pairs (IA[a], IB[b]) with IA[a] < IB[b]: a
    sample of eq. (3)'s pairs given by two lists of row indices (row blocks
    against row blocks, or one row against all others).  Same result dict as
    ``certify``."""
    X, Y = _f64(X), _f64(Y)
    n, d = X.shape
    if Y.ndim != 2 or Y.shape[0] != n:
        raise ValueError("Y must have one row per point")
    IA = np.ascontiguousarray(IA, dtype=np.int64)
    IB = np.ascontiguousarray(IB, dtype=np.int64)
    if IA.size and (IA.min() < 0 or IA.max() >= n) or IB.size and (IB.min() < 0 or IB.max() >= n):
        raise ValueError("row index out of range")
    out = OracleCert()
    _load().oracle_cross_certificate(X.ctypes.data, Y.ctypes.data, d, Y.shape[1], IA.ctypes.data, IA.shape[0],
                                     IB.ctypes.data, IB.shape[0], ctypes.byref(out))
    return {"max": out.best, "i": out.bi, "j": out.bj, "side": out.bside,
            "runner_up": out.second, "i2": out.si, "j2": out.sj, "side2": out.sside,
            "n_zero": out.nzero, "n_pairs": out.npairs}


def pair_distortions(X, Y, I, J):
    """eq. (2) for explicit pairs; -1 marks a pair of identical points."""
    X, Y = _f64(X), _f64(Y)
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    m = I.shape[0]
    out = np.empty(m, dtype=np.float64)
    side = np.empty(m, dtype=np.int32)
    _load().oracle_pair_list(X.ctypes.data, Y.ctypes.data, X.shape[1], Y.shape[1],
                             I.ctypes.data, J.ctypes.data, m, out.ctypes.data, side.ctypes.data)
    return out, side


def threads():
    """OpenMP threads the certificate loops use."""
    return int(_load().oracle_threads())


def set_threads(t):
    """Run the certificate loops on t threads from now on (t >= 1)."""
    _load().oracle_set_threads(int(t))
