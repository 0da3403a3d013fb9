"""Multicore CPU Louvain in the style of GVE-Louvain (OpenMP), used by the
benchmark as a second CPU baseline timed on all host cores.

It is neither the oracle nor part of the GPU product path: results are
checked only for validity and modularity.  ``gve_louvain.c`` holds the
algorithm; this module builds it with gcc -fopenmp and marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gve_louvain.c")
_LIB = os.path.join(_HERE, "libgve.so")
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("max_iterations", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("tol_num", ctypes.c_int64), ("tol_den", ctypes.c_int64), ("tol_drop", ctypes.c_int64),
                ("agg_num", ctypes.c_int64), ("agg_den", ctypes.c_int64)]


class _Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("iterations", ctypes.c_int32), ("moves", ctypes.c_int64),
                ("communities", ctypes.c_int64)]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gve_louvain.restype = ctypes.c_int
        lib.gve_louvain.argtypes = [ctypes.c_int64, i64p, ctypes.POINTER(ctypes.c_int32), i64p,
                                    ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(_Stats)]
        lib.gve_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().gve_max_threads())


def louvain(g, threads: int = 0, max_iterations: int = 20, max_passes: int = 10, tol_den: int = 100):
    """Run on a graphgen.CSRGraph; returns (membership int32[n], stats dict).
    Paper defaults: tau = 1/tol_den = 0.01 dropped 10x per pass, tau_agg 0.8
    (a run that continues another one after p passes starts at
    tol_den = 100 * 10^p)."""
    lib = _load()
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    w = np.ascontiguousarray(g.weights, dtype=np.int64)
    memb = np.empty(max(g.n, 1), dtype=np.int32)
    p = _Params(max_iterations, max_passes, 1, tol_den, 10, 4, 5)
    st = _Stats()
    rc = lib.gve_louvain(g.n, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         w.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(p), int(threads),
                         memb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(st))
    if rc != 0:
        raise MemoryError("gve_louvain ran out of memory")
    return memb[:g.n], {"passes": st.passes, "iterations": st.iterations, "moves": st.moves,
                        "communities": st.communities}
