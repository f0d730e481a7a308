"""MTTKRP on COO by a direct FP64 loop (oracle; test infrastructure only).

Y_n(i, r) = sum over nonzeros with i_n = i of x * prod_{m != n} A_m(i_m, r):
the element-wise form of Algorithm 1's MTTKRP step (Section III).  The loop
itself is plain C (``oracle.c``), compiled here with gcc on first use.

Pinned by: a dense unfolding times an explicit Khatri-Rao product on tiny
tensors; a single nonzero; all-ones factors (slice sums); the cross-mode
invariant <A_n, Y_n> = <X, [[A]]>.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2; OpenMP only for
    the multi-threaded timing loop)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.oracle_mttkrp_coo.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P,
                                          ctypes.c_int, ctypes.c_int, P]
        lib.oracle_mttkrp_coo.restype = ctypes.c_int
        lib.oracle_mttkrp_coo_par.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.oracle_mttkrp_coo_par.restype = ctypes.c_int
        lib.oracle_mttkrp_coo_rows.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P]
        lib.oracle_mttkrp_coo_rows.restype = ctypes.c_int
        lib.oracle_sumsq.argtypes = [ctypes.c_int64, P]
        lib.oracle_sumsq.restype = ctypes.c_double
        _lib = lib
    return _lib


def _prep(dims, inds, vals, factors, mode):
    dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int64))
    inds = np.ascontiguousarray(np.asarray(inds, dtype=np.int64))
    vals = np.ascontiguousarray(np.asarray(vals, dtype=np.float64))
    nm = dims.size
    if inds.shape != (nm, vals.size):
        raise ValueError("inds must be (N, nnz)")
    if inds.size and ((inds.min(axis=1) < 0).any() or (inds.max(axis=1) >= dims).any()):
        raise ValueError("index out of range")
    facs = []
    rank = None
    for m in range(nm):
        f = np.ascontiguousarray(np.asarray(factors[m], dtype=np.float64))
        if m != mode:
            if f.shape[0] != dims[m]:
                raise ValueError("factor %d has %d rows, dim is %d" % (m, f.shape[0], dims[m]))
            rank = f.shape[1] if rank is None else rank
            if f.shape[1] != rank:
                raise ValueError("factor ranks differ")
        facs.append(f)
    ptrs = (ctypes.c_void_p * nm)(*[f.ctypes.data for f in facs])
    return dims, inds, vals, facs, ptrs, rank


def mttkrp(dims, inds, vals, factors, mode, threads=1):
    """Y_mode (I_mode x R, float64) by the direct COO loop; threads > 1 splits
    the nonzeros over that many threads with private copies of Y (the same
    sums in another FP64 addition order)."""
    dims, inds, vals, facs, ptrs, rank = _prep(dims, inds, vals, factors, mode)
    Y = np.empty((int(dims[mode]), rank), dtype=np.float64)
    if threads > 1:
        rc = _load().oracle_mttkrp_coo_par(dims.size, dims.ctypes.data, vals.size, inds.ctypes.data,
                                           vals.ctypes.data, ptrs, rank, mode, int(threads), Y.ctypes.data)
    else:
        rc = _load().oracle_mttkrp_coo(dims.size, dims.ctypes.data, vals.size, inds.ctypes.data,
                                       vals.ctypes.data, ptrs, rank, mode, Y.ctypes.data)
    if rc:
        raise MemoryError("oracle_mttkrp_coo")
    return Y


def mttkrp_rows(dims, inds, vals, factors, mode, rows):
    """Only the listed (distinct) output rows of Y_mode, as len(rows) x R."""
    dims, inds, vals, facs, ptrs, rank = _prep(dims, inds, vals, factors, mode)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    Y = np.empty((rows.size, rank), dtype=np.float64)
    rc = _load().oracle_mttkrp_coo_rows(dims.size, dims.ctypes.data, vals.size,
                                        inds.ctypes.data, vals.ctypes.data, ptrs, rank, mode,
                                        rows.size, rows.ctypes.data, Y.ctypes.data)
    if rc == -2:
        raise ValueError("rows must be distinct and in range")
    if rc:
        raise MemoryError("oracle_mttkrp_coo_rows")
    return Y


def sumsq(vals) -> float:
    """||X||^2 = sum of squared values."""
    v = np.ascontiguousarray(np.asarray(vals, dtype=np.float64))
    return float(_load().oracle_sumsq(v.size, v.ctypes.data))
