"""ctypes front end of the C oracle (test infrastructure only).

Factors are passed as float64 copies of whatever the caller holds (FP32
factors convert exactly), values likewise, so the oracle sees exactly the
numbers the GPU path consumes and does all arithmetic in FP64.
"""

from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

from . import build as _build

_lib = None


def lib_path() -> str:
    return _build.LIB


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        f64p = ctypes.POINTER(ctypes.c_double)
        f64pp = ctypes.POINTER(f64p)
        lib.oracle_mttkrp.argtypes = [u32p, f64p, ctypes.c_uint64, ctypes.c_int, u32p, f64pp, ctypes.c_int,
                                      ctypes.c_int, f64p, ctypes.c_int]
        lib.oracle_mttkrp.restype = ctypes.c_int
        lib.oracle_mttkrp_rows.argtypes = [u32p, f64p, ctypes.c_uint64, ctypes.c_int, u32p, f64pp, ctypes.c_int,
                                           ctypes.c_int, u32p, ctypes.c_uint64, f64p]
        lib.oracle_mttkrp_rows.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prep(idx, val, dims, factors, mode):
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    if idx.ndim != 2:
        raise ValueError("idx must be (nnz, N)")
    nnz, N = idx.shape
    val = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
    if val.shape[0] != nnz:
        raise ValueError("val length must equal nnz")
    dims_a = np.ascontiguousarray(dims, dtype=np.uint32)
    if dims_a.shape[0] != N:
        raise ValueError("dims length must equal N")
    if len(factors) != N:
        raise ValueError("need one factor per mode (the output mode's entry is ignored)")
    R = None
    fac = []
    for m, f in enumerate(factors):
        if m == mode or f is None:
            fac.append(None)
            continue
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.ndim != 2 or f.shape[0] != int(dims[m]):
            raise ValueError(f"factor {m} must be ({int(dims[m])}, R)")
        if R is None:
            R = f.shape[1]
        elif f.shape[1] != R:
            raise ValueError("all factors need the same R")
        fac.append(f)
    f64p = ctypes.POINTER(ctypes.c_double)
    ptrs = (f64p * N)()
    for m, f in enumerate(fac):
        ptrs[m] = f.ctypes.data_as(f64p) if f is not None else None
    return idx, val, dims_a, fac, ptrs, nnz, N, R


def mttkrp(idx, val, dims: Sequence[int], factors, mode: int, threads: int = 1) -> np.ndarray:
    """M_mode = X_(mode) times the Khatri-Rao product of the other factors, FP64."""
    idx, val, dims_a, fac, ptrs, nnz, N, R = _prep(idx, val, dims, factors, mode)
    out = np.empty((int(dims[mode]), R), dtype=np.float64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    f64p = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_mttkrp(idx.ctypes.data_as(u32p), val.ctypes.data_as(f64p), nnz, N,
                               dims_a.ctypes.data_as(u32p), ptrs, int(mode), int(R),
                               out.ctypes.data_as(f64p), int(threads))
    if rc:
        raise ValueError(f"oracle_mttkrp failed with code {rc}")
    return out


def mttkrp_rows(idx, val, dims: Sequence[int], factors, mode: int, rows) -> np.ndarray:
    """Selected rows of M_mode, FP64 (one pass over the nonzeros)."""
    idx, val, dims_a, fac, ptrs, nnz, N, R = _prep(idx, val, dims, factors, mode)
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    out = np.empty((rows.shape[0], R), dtype=np.float64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    f64p = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_mttkrp_rows(idx.ctypes.data_as(u32p), val.ctypes.data_as(f64p), nnz, N,
                                    dims_a.ctypes.data_as(u32p), ptrs, int(mode), int(R),
                                    rows.ctypes.data_as(u32p), rows.shape[0], out.ctypes.data_as(f64p))
    if rc:
        raise ValueError(f"oracle_mttkrp_rows failed with code {rc}")
    return out


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))
