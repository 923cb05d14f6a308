"""All-core host product y = H~ x for the CPU baseline (test infrastructure:
only tests and the benchmark's cpu_baseline leg use it).

The matrix is the oracle's own CSR (``oracle.hamiltonian``); the product is a
plain-C loop over rows split across the host cores with OpenMP (spmv.c),
built by ``build_c``.  Pinned by tests/test_oracle_spmv.py against scipy's
product of the same matrix.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_spmv.so")
_lib = None


def build_c(force: bool = False) -> str:
    if force or not os.path.exists(_SO):
        subprocess.run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", _SO,
                        os.path.join(_HERE, "spmv.c")], check=True)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build_c()
        _lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        _lib.csr_matvec.argtypes = [ctypes.c_int64, P, P, P, P, P]
        _lib.csr_matvec.restype = None
        _lib.csr_threads.restype = ctypes.c_int
    return _lib


def threads() -> int:
    return int(_load().csr_threads())


def prepare(A: sp.csr_matrix):
    """(indptr int64, indices int32, data float64) of A, contiguous."""
    A = sp.csr_matrix(A)
    return (np.ascontiguousarray(A.indptr, dtype=np.int64),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64), A.shape)


def matvec(prep, x: np.ndarray, y: np.ndarray | None = None) -> np.ndarray:
    indptr, indices, data, shape = prep
    x = np.ascontiguousarray(x, dtype=np.float64)
    if y is None:
        y = np.empty(shape[0])
    _load().csr_matvec(shape[0], indptr.ctypes.data, indices.ctypes.data, data.ctypes.data,
                       x.ctypes.data, y.ctypes.data)
    return y
