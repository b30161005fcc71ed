"""ctypes access to the plain-C float64 oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_dbl_p = ctypes.POINTER(ctypes.c_double)
STATUS = {0: "ok", 1: "invalid", 2: "singular", 3: "nonfinite"}
BUILD_NOTE = _build.BUILD_NOTE


def lib():
    """The oracle library (LSE_ORACLE_LIB: another build of it, such as the
    sanitized one the CPU sanitizer test loads)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LSE_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.lse_oracle_power_sums.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            _dbl_p, _dbl_p, ctypes.c_int]
        L.lse_oracle_fit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     _dbl_p, _dbl_p, _dbl_p, _dbl_p, ctypes.c_int]
        L.lse_oracle_fit_batched.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, _dbl_p, ctypes.c_void_p, ctypes.c_int]
        L.lse_oracle_cheb_fit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          _dbl_p, _dbl_p, _dbl_p, ctypes.c_int]
        L.lse_oracle_cheb_fit_batched.argtypes = L.lse_oracle_fit_batched.argtypes
        L.lse_oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return 0
    if a.dtype == np.float64:
        return 1
    raise TypeError(f"unsupported dtype {a.dtype}")


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def power_sums(x, y, m, center=0.0, scale=1.0, threads=0):
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    S = np.zeros(2 * m + 1)
    T = np.zeros(m + 1)
    st = lib().lse_oracle_power_sums(_ptr(x), _ptr(y), x.shape[0], _dtype_code(x), m, center, scale,
                                     S.ctypes.data_as(_dbl_p), T.ctypes.data_as(_dbl_p), threads)
    if st != 0:
        raise ValueError(STATUS[st])
    return S, T


def fit(x, y, m, center=0.0, scale=1.0, threads=0) -> dict:
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    a = np.zeros(m + 1)
    b = np.zeros(m + 1)
    S = np.zeros(2 * m + 1)
    T = np.zeros(m + 1)
    st = lib().lse_oracle_fit(_ptr(x), _ptr(y), x.shape[0], _dtype_code(x), m, center, scale,
                              a.ctypes.data_as(_dbl_p), b.ctypes.data_as(_dbl_p),
                              S.ctypes.data_as(_dbl_p), T.ctypes.data_as(_dbl_p), threads)
    if st == 1:
        raise ValueError("invalid arguments")
    return {"a": a, "b": b, "S": S, "T": T, "status": STATUS[st], "center": center, "scale": scale}


def fit_batched(x, y, offsets, degrees, centers=None, scales=None, stride=None, threads=0):
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    degrees = np.ascontiguousarray(degrees, dtype=np.int32)
    B = degrees.shape[0]
    if stride is None:
        stride = int(degrees.max()) + 1 if B else 1
    a = np.full(B * stride, np.nan)
    status = np.zeros(B, dtype=np.int32)
    c = None if centers is None else np.ascontiguousarray(centers, dtype=np.float64)
    s = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
    st = lib().lse_oracle_fit_batched(_ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, _dtype_code(x),
                                      _ptr(c), _ptr(s), stride, a.ctypes.data_as(_dbl_p), _ptr(status), threads)
    if st != 0:
        raise ValueError(STATUS[st])
    return a.reshape(B, stride), status


def cheb_fit(x, y, m, center=0.0, scale=1.0, threads=0) -> dict:
    """Chebyshev coefficients c of one fit, with the Gram matrix G and D (entrywise sums)."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    c = np.zeros(m + 1)
    G = np.zeros((m + 1, m + 1))
    D = np.zeros(m + 1)
    st = lib().lse_oracle_cheb_fit(_ptr(x), _ptr(y), x.shape[0], _dtype_code(x), m, center, scale,
                                   c.ctypes.data_as(_dbl_p), G.ctypes.data_as(_dbl_p), D.ctypes.data_as(_dbl_p),
                                   threads)
    if st == 1:
        raise ValueError("invalid arguments")
    return {"c": c, "G": G, "D": D, "status": STATUS[st], "center": center, "scale": scale}


def cheb_fit_batched(x, y, offsets, degrees, centers=None, scales=None, stride=None, threads=0):
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y, dtype=x.dtype)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    degrees = np.ascontiguousarray(degrees, dtype=np.int32)
    B = degrees.shape[0]
    if stride is None:
        stride = int(degrees.max()) + 1 if B else 1
    out = np.full(B * stride, np.nan)
    status = np.zeros(B, dtype=np.int32)
    c = None if centers is None else np.ascontiguousarray(centers, dtype=np.float64)
    s = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
    st = lib().lse_oracle_cheb_fit_batched(_ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, _dtype_code(x),
                                           _ptr(c), _ptr(s), stride, out.ctypes.data_as(_dbl_p), _ptr(status),
                                           threads)
    if st != 0:
        raise ValueError(STATUS[st])
    return out.reshape(B, stride), status


def max_threads() -> int:
    return int(lib().lse_oracle_max_threads())
