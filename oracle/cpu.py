"""ctypes wrapper of the C oracle (TEST INFRASTRUCTURE ONLY).

Same float64 definitions as `ref`, as plain parallel C loops, for sizes where
NumPy is too slow.  Loads oracle/liborc.so, building it with gcc if absent.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Sequence, Tuple

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_max_threads.restype = C.c_int
        L.orc_mttkrp.restype = C.c_int
        L.orc_mttkrp.argtypes = [C.c_int, C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_void_p),
                                 C.c_void_p, C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_void_p,
                                 C.c_int]
        L.orc_ttm_group.restype = C.c_int64
        L.orc_ttm_group.argtypes = [C.c_int, C.c_int64, C.POINTER(C.c_void_p), C.c_int, C.c_void_p,
                                    C.c_void_p]
        L.orc_ttm.restype = C.c_int
        L.orc_ttm.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        L.orc_model.restype = C.c_int
        L.orc_model.argtypes = [C.c_int, C.c_int64, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                C.c_int, C.c_void_p, C.c_int]
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _ptrs(arrs):
    return (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])


def _prep(dims, idx, vals, factors):
    idx = [np.ascontiguousarray(i, dtype=np.int32) for i in idx]
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    factors = [np.ascontiguousarray(f, dtype=np.float64) for f in factors] if factors is not None else None
    d = (C.c_int64 * len(dims))(*[int(x) for x in dims])
    return d, idx, vals, factors


def mttkrp(dims, idx, vals, factors, mode, nthreads=0, return_threads=False):
    """Eq. (6) over the nonzeros, float64; returns M (dims[mode] x R)."""
    d, idx, vals, factors = _prep(dims, idx, vals, factors)
    R = factors[0].shape[1]
    out = np.zeros((int(dims[mode]), R), dtype=np.float64)
    t = lib().orc_mttkrp(len(dims), d, int(vals.shape[0]), _ptrs(idx), vals.ctypes.data,
                         _ptrs(factors), R, int(mode), out.ctypes.data, int(nthreads))
    if t < 0:
        raise MemoryError("orc_mttkrp")
    return (out, t) if return_threads else out


def ttm_group(dims, idx, mode) -> Tuple[np.ndarray, np.ndarray]:
    """Grouping pass for SpTTM: (nonzero ids grouped by fibre, fibre pointers)."""
    idx = [np.ascontiguousarray(i, dtype=np.int32) for i in idx]
    Z = idx[0].shape[0]
    order = np.empty(Z, dtype=np.int64)
    ptr = np.empty(Z + 1, dtype=np.int64)
    nf = lib().orc_ttm_group(len(dims), Z, _ptrs(idx), int(mode), order.ctypes.data, ptr.ctypes.data)
    return order, ptr[:nf + 1].copy()


def ttm(dims, idx, vals, U, mode, group=None, nthreads=0, return_threads=False):
    """Eq. (3) over the nonzeros, float64; returns (fibres[nfib, N-1], Y[nfib, R])."""
    idx = [np.ascontiguousarray(i, dtype=np.int32) for i in idx]
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    order, ptr = group if group is not None else ttm_group(dims, idx, mode)
    nf = ptr.shape[0] - 1
    R = U.shape[1]
    Y = np.empty((nf, R), dtype=np.float64)
    t = lib().orc_ttm(nf, order.ctypes.data, ptr.ctypes.data, idx[mode].ctypes.data,
                      vals.ctypes.data, U.ctypes.data, R, Y.ctypes.data, int(nthreads))
    imodes = [m for m in range(len(dims)) if m != mode]
    first = order[ptr[:-1]]
    fibres = np.stack([idx[m][first].astype(np.int64) for m in imodes], axis=1) if nf else \
        np.zeros((0, len(dims) - 1), np.int64)
    return (fibres, Y, t) if return_threads else (fibres, Y)


def model_at(idx, factors, nthreads=0) -> np.ndarray:
    idx = [np.ascontiguousarray(i, dtype=np.int32) for i in idx]
    factors = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    Z = idx[0].shape[0]
    out = np.empty(Z, dtype=np.float64)
    lib().orc_model(len(idx), Z, _ptrs(idx), _ptrs(factors), factors[0].shape[1], out.ctypes.data,
                    int(nthreads))
    return out


def model_adjoint(dims, idx, g, factors, nthreads=0) -> List[np.ndarray]:
    """Chain-rule gradient of sum_e g_e xhat_e: Eq. (6) with values g, per mode."""
    return [mttkrp(dims, idx, g, factors, m, nthreads) for m in range(len(dims))]


def mse_grad(dims, idx, vals, factors, nthreads=0) -> Tuple[float, List[np.ndarray]]:
    Z = len(vals)
    r = model_at(idx, factors, nthreads) - np.asarray(vals, np.float64)
    loss = float(0.5 * np.dot(r, r) / Z)
    return loss, model_adjoint(dims, idx, r / Z, factors, nthreads)
