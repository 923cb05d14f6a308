"""Basis sampling (Sec. Subspace of the ground state; Sec. Other sampling
methods).

The truncated basis F~ of the benchmark workloads is drawn by a Metropolis
chain: one random hop per step (the paper's variant 2 proposal), accepted
with the ratio of Boltzmann factors of the diagonal energy (variant 1, Eq.
boltzmann_factor2, with U n_U generalised to the full diagonal energy and
inverse temperature beta_s).  The exact stream is specified in chain.c.

``chain_python`` is a pure-Python loop for small cases; ``chain_c`` calls the
plain-C version (built by ``build_c``).  The two are pinned against each other
bit for bit, and the C chain's visit frequencies are pinned against the exact
stationary distribution exp(-beta_s E_diag)/Z on enumerated sectors
(detailed balance of a symmetric proposal with Metropolis acceptance).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_chain.so")
_lib = None

MASK = (1 << 64) - 1


def build_c(force: bool = False) -> str:
    src = os.path.join(_HERE, "chain.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-shared", "-fPIC",
                               "-o", _SO, src, "-lm"])
    return _SO


def _load():
    global _lib
    if _lib is None:
        build_c()
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        lib.oracle_chain.restype = ctypes.c_int64
        lib.oracle_chain.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int),
                                     P(ctypes.c_double), P(ctypes.c_double), ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_double, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, P(ctypes.c_uint64),
                                     P(ctypes.c_int64)]
        lib.oracle_chain_histogram.restype = ctypes.c_int
        lib.oracle_chain_histogram.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int),
                                               P(ctypes.c_double), P(ctypes.c_double),
                                               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                               ctypes.c_int64, ctypes.c_int64, P(ctypes.c_uint64),
                                               ctypes.c_int64, P(ctypes.c_int64)]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _bond_ij(model):
    bi = np.array([b[0] for b in model.bonds], dtype=np.int32)
    bj = np.array([b[1] for b in model.bonds], dtype=np.int32)
    return bi, bj


def chain_c(model, start: int, seed: int, n_f: int, burn_in: int, max_steps: int,
            beta_s: float = 0.5):
    """Sorted distinct keys of the chain and the number of steps taken."""
    lib = _load()
    bi, bj = _bond_ij(model)
    U = np.ascontiguousarray(model.U, dtype=np.float64)
    eps = np.ascontiguousarray(model.eps, dtype=np.float64)
    out = np.zeros(n_f, dtype=np.uint64)
    steps = ctypes.c_int64(0)
    k = lib.oracle_chain(len(bi), _ptr(bi, ctypes.c_int), _ptr(bj, ctypes.c_int),
                         _ptr(U, ctypes.c_double), _ptr(eps, ctypes.c_double),
                         ctypes.c_uint64(start), ctypes.c_uint64(seed), beta_s,
                         burn_in, max_steps, n_f, _ptr(out, ctypes.c_uint64),
                         ctypes.byref(steps))
    if k < 0:
        raise MemoryError("oracle chain: allocation failed")
    return out[:k].copy(), int(steps.value)


def chain_histogram(model, start, seed, burn_in, steps, keys, beta_s=0.5):
    lib = _load()
    bi, bj = _bond_ij(model)
    U = np.ascontiguousarray(model.U, dtype=np.float64)
    eps = np.ascontiguousarray(model.eps, dtype=np.float64)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    counts = np.zeros(len(keys), dtype=np.int64)
    rc = lib.oracle_chain_histogram(len(bi), _ptr(bi, ctypes.c_int), _ptr(bj, ctypes.c_int),
                                    _ptr(U, ctypes.c_double), _ptr(eps, ctypes.c_double),
                                    ctypes.c_uint64(start), ctypes.c_uint64(seed), beta_s,
                                    burn_in, steps, _ptr(keys, ctypes.c_uint64), len(keys),
                                    _ptr(counts, ctypes.c_int64))
    if rc != 0:
        raise RuntimeError("chain left the enumerated sector")
    return counts


def chain_python(model, start: int, seed: int, n_f: int, burn_in: int, max_steps: int,
                 beta_s: float = 0.5):
    """Pure-Python loop of the same chain (small cases only)."""
    state = seed & MASK

    def nxt():
        nonlocal state
        state = (state + 0x9E3779B97F4A7C15) & MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    spins = [start >> 32, start & 0xFFFFFFFF]
    M = 4 * len(model.bonds)
    seen = set()
    step = 0
    while step < max_steps and len(seen) < n_f:
        r0, r1 = nxt(), nxt()
        m = ((r0 >> 32) * M) >> 32
        b, spin, d = m >> 2, (m >> 1) & 1, m & 1
        i, j = sorted(model.bonds[b][:2])
        src, dst = (i, j) if d == 0 else (j, i)
        s, o = spins[spin], spins[1 - spin]
        if (s >> src) & 1 and not (s >> dst) & 1:
            dE = (model.eps[dst] - model.eps[src]) + (model.U[dst] * float((o >> dst) & 1)
                                                      - model.U[src] * float((o >> src) & 1))
            u = (r1 >> 11) * (1.0 / 9007199254740992.0)
            if dE <= 0.0 or u < math.exp(-beta_s * dE):
                spins[spin] = s ^ ((1 << src) | (1 << dst))
        step += 1
        if step > burn_in:
            seen.add((spins[0] << 32) | spins[1])
    return np.array(sorted(seen), dtype=np.uint64), step
