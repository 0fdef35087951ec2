"""ctypes front of the C oracle (oracle/scan.c): the plain O(n^2) method.

TEST INFRASTRUCTURE, like everything under oracle/: only tests, the smoke
check and the benchmark's CPU baseline use it.  It builds its own library with
gcc (no HIP) and shares nothing with the product library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .dpc_oracle import cutoff_square

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scan.c")
_LIB = os.path.join(_HERE, "liboracle_scan.so")
_lib = None

_I32P = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def build(force: bool = True) -> str:
    """Compile scan.c into liboracle_scan.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_rho.argtypes = [_I32P, _I64, _I32, _I64, _I32P]
        lib.oracle_rho_of.argtypes = [_I32P, _I64, _I32, _I64, _I64P, _I64, _I32P]
        lib.oracle_order.argtypes = [_I32P, _I64, _I64P]
        lib.oracle_dependent.argtypes = [_I32P, _I64, _I32, _I32P, _I32P, _I64P]
        lib.oracle_dependent_of.argtypes = [_I32P, _I64, _I32, _I64, _I64P, _I64, _I64, _I32P, _I32P, _I64P]
        lib.oracle_delta.argtypes = [_I64P, _I64, _F64P]
        lib.oracle_labels.argtypes = [_I32P, _I32P, _F64P, _I64, _I32, ctypes.c_double, _I32P]
        lib.oracle_labels.restype = _I64
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def _pts(pts) -> np.ndarray:
    p = np.ascontiguousarray(pts, dtype=np.int32)
    if p.ndim != 2:
        raise ValueError("points must be [n, d]")
    return p


def local_density(pts, d_cut: float) -> np.ndarray:
    p = _pts(pts)
    rho = np.empty(p.shape[0], np.int32)
    _load().oracle_rho(p, p.shape[0], p.shape[1], cutoff_square(d_cut), rho)
    return rho


def local_density_of(pts, d_cut: float, which) -> np.ndarray:
    p = _pts(pts)
    w = np.ascontiguousarray(which, dtype=np.int64)
    out = np.empty(w.size, np.int32)
    _load().oracle_rho_of(p, p.shape[0], p.shape[1], cutoff_square(d_cut), w, w.size, out)
    return out


def density_order(rho) -> np.ndarray:
    r = np.ascontiguousarray(rho, dtype=np.int32)
    order = np.empty(r.size, np.int64)
    _load().oracle_order(r, r.size, order)
    return order


def dependent(pts, rho) -> tuple[np.ndarray, np.ndarray]:
    p = _pts(pts)
    r = np.ascontiguousarray(rho, dtype=np.int32)
    dep = np.empty(p.shape[0], np.int32)
    d2 = np.empty(p.shape[0], np.int64)
    _load().oracle_dependent(p, p.shape[0], p.shape[1], r, dep, d2)
    return dep, d2


def dependent_of(pts, d_cut: float, which, max_walk: int = 0):
    """(rho, dep, d2) of the listed points only; dep = -2 if undecided in max_walk."""
    p = _pts(pts)
    w = np.ascontiguousarray(which, dtype=np.int64)
    rho = np.empty(w.size, np.int32)
    dep = np.empty(w.size, np.int32)
    d2 = np.empty(w.size, np.int64)
    _load().oracle_dependent_of(p, p.shape[0], p.shape[1], cutoff_square(d_cut), w, w.size,
                                int(max_walk), rho, dep, d2)
    return rho, dep, d2


def dependent_distance(d2) -> np.ndarray:
    x = np.ascontiguousarray(d2, dtype=np.int64)
    out = np.empty(x.size, np.float64)
    _load().oracle_delta(x, x.size, out)
    return out


def labels(rho, dep, delta, rho_min: int, delta_min: float) -> tuple[np.ndarray, int]:
    r = np.ascontiguousarray(rho, dtype=np.int32)
    q = np.ascontiguousarray(dep, dtype=np.int32)
    dl = np.ascontiguousarray(delta, dtype=np.float64)
    lab = np.empty(r.size, np.int32)
    nc = _load().oracle_labels(r, q, dl, r.size, int(rho_min), float(delta_min), lab)
    return lab, int(nc)


def dpc(pts, d_cut: float, rho_min: int, delta_min: float) -> dict:
    rho = local_density(pts, d_cut)
    dep, d2 = dependent(pts, rho)
    delta = dependent_distance(d2)
    lab, nc = labels(rho, dep, delta, rho_min, delta_min)
    return {"rho": rho, "dep": dep, "d2": d2, "delta": delta, "label": lab, "ncenters": nc}
