"""Fock states of one (N_up, N_dn) sector.

A Fock state is stored as key = (up << 32) | down with site i <-> bit i of
each spin string (the paper writes the up string first, App. BFS vs DFS).
The sector of fixed N_e and S_z has C(Nc, N_up) * C(Nc, N_dn) states
(Sec. Exact diagonalization).

Pins: sector sizes against binomials and the paper's 36-state 4-site sector
(App. BFS vs DFS), 165,636,900 = C(16,8)^2 (Table reduce_green).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)


def strings(n_orb: int, n_el: int) -> np.ndarray:
    """All occupation strings of n_el electrons in n_orb orbitals, ascending."""
    out = [sum(1 << i for i in c) for c in itertools.combinations(range(n_orb), n_el)]
    return np.array(sorted(out), dtype=np.uint64)


def sector_keys(n_orb: int, n_up: int, n_dn: int) -> np.ndarray:
    """Every key of the sector, sorted ascending (up string major)."""
    ups = strings(n_orb, n_up)
    dns = strings(n_orb, n_dn)
    keys = (ups[:, None] << np.uint64(32)) | dns[None, :]
    return np.sort(keys.ravel())


def sector_size(n_orb: int, n_up: int, n_dn: int) -> int:
    return math.comb(n_orb, n_up) * math.comb(n_orb, n_dn)


def split(keys: np.ndarray):
    keys = np.asarray(keys, dtype=np.uint64)
    return keys >> np.uint64(32), keys & MASK32


def bit(s: np.ndarray, i: int) -> np.ndarray:
    return ((s >> np.uint64(i)) & np.uint64(1)).astype(np.int64)


def double_occupation(keys: np.ndarray) -> np.ndarray:
    """n_U = sum_i n_{i up} n_{i dn} (the paper's n_U definition)."""
    up, dn = split(keys)
    return np.bitwise_count(up & dn).astype(np.int64)


def diagonal(keys: np.ndarray, model) -> np.ndarray:
    """<x|H|x> = sum_i U_i n_iu n_id + sum_{i s} eps_i n_is, term by term."""
    up, dn = split(keys)
    d = np.zeros(len(keys), dtype=np.float64)
    for i in range(model.n_orb):
        nu, nd = bit(up, i), bit(dn, i)
        d += model.U[i] * (nu * nd)
        d += model.eps[i] * (nu + nd)
    return d


def check_sector(keys: np.ndarray, model) -> None:
    """Keys must be sorted, unique, inside n_orb bits and in the sector."""
    keys = np.asarray(keys, dtype=np.uint64)
    up, dn = split(keys)
    assert np.all(keys[1:] > keys[:-1])
    assert np.all(np.bitwise_count(up) == model.n_up)
    assert np.all(np.bitwise_count(dn) == model.n_dn)
    lim = np.uint64((1 << model.n_orb) - 1) if model.n_orb < 64 else None
    assert np.all((up & ~lim) == 0) and np.all((dn & ~lim) == 0)
