"""Build and load the plain-C part of the oracle (test infrastructure only).

The C source is compiled with gcc (no fast-math, IEEE FP64 on SSE2) into
``oracle/_tsdf_oracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "tsdf_oracle.c")
LIB = os.path.join(_HERE, "_tsdf_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        f = ctypes.c_float
        L.oracle_walk.argtypes = [P, P, d, P, P, i64, P, P, P, P]
        L.oracle_ray_range.argtypes = [P, P, d, P, P, i64, P, P]
        L.oracle_integrate.argtypes = [P, P, d, d, P, P, P, i64, P, P, d, P, P, P]
        L.oracle_bounds.argtypes = [P, P, d, ctypes.c_int32, P, P, P, i64, f, P, P, P, P, P, P]
        for fn in (L.oracle_walk, L.oracle_ray_range, L.oracle_integrate, L.oracle_bounds):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib
