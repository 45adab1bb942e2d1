"""ctypes loader for the oracle's C Slater-Condon core (``sc.c``).

Test infrastructure only.  The library is compiled with gcc on first use (or
by ``build()``) into ``oracle/liboracle_sc.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc.c")
_LIB = os.path.join(_HERE, "liboracle_sc.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``sc.c`` with gcc into ``liboracle_sc.so`` (always when ``force``)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        ip64 = ctypes.POINTER(ctypes.c_int64)
        ip32 = ctypes.POINTER(ctypes.c_int32)
        L.sc_element.restype = ctypes.c_double
        L.sc_element.argtypes = [ctypes.c_int, dp, dp, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64]
        L.sc_build_csr.restype = ctypes.c_int64
        L.sc_build_csr.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int, up,
                                   ctypes.c_int, up, ip64, ip32, dp]
        L.sc_diagonal.restype = None
        L.sc_diagonal.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int, up,
                                  ctypes.c_int, up, dp]
        L.sc_sigma_rows.restype = None
        L.sc_sigma_rows.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int, up,
                                    ctypes.c_int, up, dp, ctypes.c_int, ip64, dp]
        L.sc_direct_setup.restype = ctypes.c_void_p
        L.sc_direct_setup.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, up, ctypes.c_int, up, dp]
        L.sc_direct_free.restype = None
        L.sc_direct_free.argtypes = [ctypes.c_void_p]
        L.sc_direct_sigma.restype = None
        L.sc_direct_sigma.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_int, ctypes.c_int]
        L.sc_rdm12.restype = None
        L.sc_rdm12.argtypes = [ctypes.c_int, ctypes.c_int, up, ctypes.c_int, up, dp, dp, dp]
        _lib = L
    return _lib


def ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)
