"""Oracle step O6: no-pivot banded LU of every A_j, and local solves.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The arithmetic lives in the plain C file ``bandlu.c`` (loops written out);
this module converts CSR matrices to band storage, compiles the C file with
gcc when its shared object is missing or older than the source, and calls it
through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bandlu.c")
_SO = os.path.join(_HERE, "_bandlu.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile bandlu.c with gcc (plain -O2, OpenMP over matrices)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        _lib.oracle_band_lu.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_double, P]
        _lib.oracle_band_lu.restype = ctypes.c_int
        _lib.oracle_band_solve.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        _lib.oracle_band_lu_batch.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
        _lib.oracle_band_solve_batch.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_int]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


_threads = None


def set_threads(n=None):
    """Host threads of the batched factorisation and solves (None: up to 16)."""
    global _threads
    _threads = None if n is None else max(1, int(n))


def nthreads() -> int:
    if _threads is not None:
        return _threads
    return max(1, min(16, os.cpu_count() or 1))


def to_band(A, b: int) -> np.ndarray:
    """CSR/COO -> band array (n, 2b+1), entry (r, c) at [r, b + c - r]."""
    A = A.tocoo()
    n = A.shape[0]
    AB = np.zeros((n, 2 * b + 1), dtype=np.complex128)
    d = A.col - A.row
    if np.any(np.abs(d) > b):
        raise ValueError("matrix is wider than the band")
    np.add.at(AB, (A.row, b + d), A.data)
    return AB


def band_lu(AB: np.ndarray, b: int, tol_abs: float = 0.0):
    """In-place no-pivot LU; returns (status, max|U|)."""
    AB = np.ascontiguousarray(AB, dtype=np.complex128)
    mu = ctypes.c_double(0.0)
    st = lib().oracle_band_lu(AB.shape[0], b, _ptr(AB), tol_abs, ctypes.byref(mu))
    return AB, st, mu.value


def band_solve(LU: np.ndarray, b: int, rhs: np.ndarray) -> np.ndarray:
    x = np.array(rhs, dtype=np.complex128, copy=True)
    lib().oracle_band_solve(LU.shape[0], b, _ptr(LU), _ptr(x))
    return x


def unpack_lu(LU: np.ndarray, b: int):
    """Dense (L, U) from the in-place band factors (small matrices only)."""
    n = LU.shape[0]
    L = np.eye(n, dtype=np.complex128)
    U = np.zeros((n, n), dtype=np.complex128)
    for r in range(n):
        for c in range(max(0, r - b), min(n, r + b + 1)):
            v = LU[r, b + c - r]
            if c < r:
                L[r, c] = v
            else:
                U[r, c] = v
    return L, U


class BandBatch:
    """All local factorisations of one problem, stored back to back."""

    def __init__(self, mats, bands, tol_rel: float = 1e-14):
        self.n = np.array([m.shape[0] for m in mats], dtype=np.int32)
        self.b = np.array(bands, dtype=np.int32)
        w = 2 * self.b.astype(np.int64) + 1
        sizes = self.n.astype(np.int64) * w
        self.off = np.zeros(len(mats), dtype=np.int64)
        self.off[1:] = np.cumsum(sizes)[:-1]
        self.data = np.zeros(int(sizes.sum()), dtype=np.complex128)
        amax = np.zeros(len(mats))
        for m, (A, b) in enumerate(zip(mats, bands)):
            AB = to_band(A, int(b))
            amax[m] = np.abs(AB).max() if AB.size else 0.0
            self.data[self.off[m]:self.off[m] + AB.size] = AB.ravel()
        self.amax = amax
        tol = (tol_rel * amax).astype(np.float64)
        self.status = np.zeros(len(mats), dtype=np.int32)
        self.max_u = np.zeros(len(mats), dtype=np.float64)
        lib().oracle_band_lu_batch(len(mats), _ptr(self.n), _ptr(self.b), _ptr(self.off),
                                   _ptr(self.data), _ptr(tol), _ptr(self.status),
                                   _ptr(self.max_u), nthreads())
        self.voff = np.zeros(len(mats), dtype=np.int64)
        self.voff[1:] = np.cumsum(self.n.astype(np.int64))[:-1]
        self.nloc = int(self.n.astype(np.int64).sum())

    def factors(self, m: int) -> np.ndarray:
        n, b = int(self.n[m]), int(self.b[m])
        return self.data[self.off[m]:self.off[m] + n * (2 * b + 1)].reshape(n, 2 * b + 1)

    def growth(self) -> np.ndarray:
        """Pivot growth max|U| / max|A| per matrix."""
        return self.max_u / np.where(self.amax > 0, self.amax, 1.0)

    def solve_all(self, vec: np.ndarray) -> np.ndarray:
        """vec holds every local right-hand side back to back (voff)."""
        x = np.ascontiguousarray(vec, dtype=np.complex128).copy()
        lib().oracle_band_solve_batch(len(self.n), _ptr(self.n), _ptr(self.b), _ptr(self.off),
                                      _ptr(self.data), _ptr(self.voff), _ptr(x), nthreads())
        return x
