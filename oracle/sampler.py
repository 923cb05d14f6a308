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

The paper's step sampler (``bfs_python`` / ``bfs_numpy``, Eq.
boltzmann_factor) is pinned by: the two forms bit for bit; its limits (beta = 0
reaches the whole sector in breadth-first shells, large beta keeps only states
without double occupation); the sizes of the pre-accepted levels; and the
acceptance law itself -- over many seeds, the kept fraction of first-step
proposals with n_U = 0, 1, 2 matches min(1, exp(-beta U n_U)) at two values of
U (a law without U, or one taken on the change of n_U, is rejected).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import fock

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


# ---------------------------------------------------------------------------
# The paper's MCD sampler (Sec. Subspace of the ground state, the numbered
# "step" procedure and Eq. boltzmann_factor).
#
# Reading used (the paper leaves the RNG and tie-breaks open):
#  * a step takes the frontier (the states accepted in the previous step)
#    in ascending key order and applies every hop to each parent, hops in
#    the order (bond, spin up then down, direction i->j then j->i), i.e. hop
#    index h in [0, 4 n_bonds) with bond h >> 2, spin (h >> 1) & 1, dir h & 1;
#  * a possible hop is accepted with probability min(exp(-beta U n_U), 1),
#    where U is the (uniform) on-site repulsion of the orbitals with U != 0
#    and n_U the double occupation of the proposed state on those orbitals;
#    the uniform number is u = (z >> 11) 2^-53 with
#    z = f(f(f(seed ^ (step * G)) ^ parent) ^ h), f(x) = the splitmix64
#    output function applied to x + G, G = 0x9E3779B97F4A7C15;
#  * the next frontier is every accepted proposal (new or already in F~),
#    each state once; accepted proposals are ordered by (parent rank, h) and
#    a state keeps its first occurrence;
#  * new states join F~ in that order; the sampling stops as soon as F~
#    holds n_f states (mid-step), or after max_steps steps;
#  * an empty frontier is refilled with all of F~.
#  * pre-acceptance (Sec. Monte Carlo sampling, last paragraph): with a level
#    L > 0 every sector state with n_U < L is accepted before the search
#    (F~ and the first frontier are that set, the start state is not used),
#    so the search only has to find states of the remaining n_U; if that set
#    already holds >= n_f states, F~ is its first n_f states in (n_U, key)
#    order and no step is taken.  Reading: every orbital is interacting (one
#    common U), as in the paper's lattice clusters.
# ---------------------------------------------------------------------------
G64 = 0x9E3779B97F4A7C15


def _f64(x):
    z = (x + G64) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def _uniform_u(seed, step, parent, h):
    z = _f64((seed ^ ((step * G64) & MASK)) & MASK)
    z = _f64(z ^ parent)
    z = _f64(z ^ h)
    return (z >> 11) * (1.0 / 9007199254740992.0)


def _u_and_table(model, beta):
    us = sorted(set(float(u) for u in model.U if u != 0.0))
    if len(us) > 1:
        raise ValueError("BFS sampler needs one common U on the interacting orbitals")
    U0 = us[0] if us else 0.0
    umask = sum(1 << i for i in range(model.n_orb) if model.U[i] != 0.0)
    table = [math.exp(-beta * U0 * k) for k in range(model.n_orb + 1)]
    return umask, table


def preaccepted(model, level):
    """Sector states with fewer than `level` doubly occupied orbitals, in
    (n_U, key) order (brute force over the enumerated sector)."""
    if level <= 0:
        return np.zeros(0, dtype=np.uint64)
    if any(u == 0.0 for u in model.U):
        raise ValueError("pre-acceptance needs U != 0 on every orbital")
    keys = fock.sector_keys(model.n_orb, model.n_up, model.n_dn)
    nu = fock.double_occupation(keys)
    sel = nu < level
    order = np.lexsort((keys[sel], nu[sel]))
    return keys[sel][order]


def _initial(model, start, n_f, level):
    """(F~, frontier, done) at the start of the search."""
    P = preaccepted(model, level)
    if len(P) == 0:
        return [int(start)], [int(start)], False
    if len(P) >= n_f:
        return [int(k) for k in P[:n_f]], [], True
    return [int(k) for k in P], sorted(int(k) for k in P), False


def bfs_python(model, start, seed, beta, n_f, max_steps, pre_level=0):
    """Plain-loop implementation of the MCD step sampler (small cases)."""
    umask, table = _u_and_table(model, beta)
    bonds = [tuple(sorted(b[:2])) for b in model.bonds]
    H = 4 * len(bonds)
    S, F, done = _initial(model, start, n_f, pre_level)
    if done:
        return np.array(sorted(S), dtype=np.uint64), 0
    inS = set(S)
    step = 0
    while len(S) < n_f and step < max_steps:
        step += 1
        if not F:
            F = sorted(S)
        F = sorted(F)
        seen = {}
        order = []
        for rank, x in enumerate(F):
            up, dn = x >> 32, x & 0xFFFFFFFF
            for h in range(H):
                i, j = bonds[h >> 2]
                spin, d = (h >> 1) & 1, h & 1
                src, dst = (i, j) if d == 0 else (j, i)
                s = up if spin == 0 else dn
                if not ((s >> src) & 1) or ((s >> dst) & 1):
                    continue
                s2 = s ^ ((1 << src) | (1 << dst))
                y = (s2 << 32) | dn if spin == 0 else (up << 32) | s2
                nu = bin((y >> 32) & y & umask).count("1")
                if _uniform_u(seed, step, x, h) < table[nu]:
                    if y not in seen:
                        seen[y] = len(order)
                        order.append(y)
        for y in order:
            if y not in inS:
                S.append(y)
                inS.add(y)
                if len(S) >= n_f:
                    break
        F = order
    return np.array(sorted(S), dtype=np.uint64), step


def bfs_numpy(model, start, seed, beta, n_f, max_steps, pre_level=0):
    """Vectorised implementation of the same sampler (one step = array ops)."""
    umask, table = _u_and_table(model, beta)
    table = np.array(table)
    bi = np.array([min(b[0], b[1]) for b in model.bonds], dtype=np.uint64)
    bj = np.array([max(b[0], b[1]) for b in model.bonds], dtype=np.uint64)
    H = 4 * len(bi)
    h = np.arange(H, dtype=np.uint64)
    hb = (h >> np.uint64(2)).astype(np.int64)
    spin = (h >> np.uint64(1)) & np.uint64(1)
    d = h & np.uint64(1)
    src = np.where(d == 0, bi[hb], bj[hb])
    dst = np.where(d == 0, bj[hb], bi[hb])
    one = np.uint64(1)
    S0, F0, done = _initial(model, start, n_f, pre_level)
    S = np.array(S0, dtype=np.uint64)
    F = np.array(F0, dtype=np.uint64)
    if done:
        return np.sort(S), 0
    step = 0
    with np.errstate(over="ignore"):
        while len(S) < n_f and step < max_steps:
            step += 1
            if len(F) == 0:
                F = np.sort(S)
            F = np.sort(F)
            up = (F >> np.uint64(32))[:, None]
            dn = (F & np.uint64(0xFFFFFFFF))[:, None]
            s = np.where(spin[None, :] == 0, up, dn)
            ok = (((s >> src[None, :]) & one) == 1) & (((s >> dst[None, :]) & one) == 0)
            s2 = s ^ ((one << src[None, :]) | (one << dst[None, :]))
            y = np.where(spin[None, :] == 0, (s2 << np.uint64(32)) | dn, (up << np.uint64(32)) | s2)
            nu = np.bitwise_count((y >> np.uint64(32)) & y & np.uint64(umask)).astype(np.int64)
            # counter-based uniforms
            G = np.uint64(G64)
            def f(x):
                z = x + G
                z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
                z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
                return z ^ (z >> np.uint64(31))
            z0 = f(np.uint64(seed) ^ (np.uint64(step) * G))
            z = f(f(z0 ^ F[:, None]) ^ h[None, :])
            u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
            acc = ok & (u < table[nu])
            ys = y[acc]                          # row-major = (parent rank, h) order
            if len(ys) == 0:
                F = ys
                continue
            uniq, first = np.unique(ys, return_index=True)
            order = uniq[np.argsort(first, kind="stable")]
            new = order[~np.isin(order, S)]
            room = n_f - len(S)
            S = np.concatenate([S, new[:room]])
            F = order
    return np.sort(S), step
