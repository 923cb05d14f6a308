"""Lanczos ground state (App. Lanczos).

Recurrence (Eq. next_vector, Eq. an_bn): phi_{n+1} = H phi_n - a_n phi_n -
b_n phi_{n-1} with a_n = <phi_n|H|phi_n>/<phi_n|phi_n> and
b_n^2 = <phi_n|phi_n>/<phi_{n-1}|phi_{n-1}>, b_0 = 0, phi_{-1} = 0.  The paper
normalises |n> = |phi_n>/<phi_n|phi_n>, a garbled square root: the reading
used here is the orthonormal basis |n> = |phi_n>/||phi_n||, for which the
tridiagonal H_eff has a_n on the diagonal and b_n = ||phi_n||/||phi_{n-1}||
off it.  The ground state is rebuilt as |Omega> = sum_n |n><n|Omega_eff>
(Eq. change_basis).

The oracle keeps every Krylov vector and reorthogonalises fully (twice,
classical Gram-Schmidt), then takes |Omega> from the stored vectors; the
second-pass reconstruction of Eq. change_basis is also provided
(``recompute_ground_state``) and pinned against the stored form.

Start vector (the paper only says "random"): phi_0[n] = 2u - 1 with u the
top 53 bits of the first splitmix64 output of the state (seed XOR key_n),
so the vector depends only on the keys and the seed.

Convergence reading: stop when the Ritz residual b_{k+1} |s_k| of the lowest
Ritz pair is <= tol * max(1, |E0|), or on breakdown (b_{k+1} ~ 0).

Pins: tests/test_oracle_lanczos.py (2-site closed form, free fermions at
U = 0, dense eigh on full sectors, the paper's full-ED energy tables).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_first(state: np.ndarray) -> np.ndarray:
    """First output of Vigna's splitmix64 generator started at `state`."""
    with np.errstate(over="ignore"):
        z = np.asarray(state, dtype=np.uint64) + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def start_vector(keys: np.ndarray, seed: int) -> np.ndarray:
    z = splitmix64_first(np.asarray(keys, dtype=np.uint64) ^ np.uint64(seed))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def _lowest(alpha, beta):
    if len(alpha) == 1:
        return alpha[0], np.ones(1)
    w, s = eigh_tridiagonal(np.asarray(alpha), np.asarray(beta), select="i",
                            select_range=(0, 0))
    return w[0], s[:, 0]


def lanczos_ground(H, phi0: np.ndarray, tol: float = 1e-12, max_iter: int = 400,
                   reorth: bool = True, min_iter: int = 1, keep_vectors: bool = True):
    """Lowest eigenpair of the symmetric operator H (matrix or callable).

    Returns dict(e0, psi0, alpha, beta, iters, residual).  keep_vectors=False
    (no reorthogonalisation only) keeps just the last two Krylov vectors, the
    recurrence unchanged, and returns psi0 = None (Eq. change_basis can then
    be taken by ``recompute_ground_state``): for bases whose Krylov store
    would not fit in host memory.
    """
    if not keep_vectors and reorth:
        raise ValueError("full reorthogonalisation needs the stored vectors")
    mv = H if callable(H) else (lambda x: H @ x)
    n = len(phi0)
    v = phi0 / np.linalg.norm(phi0)
    V = [v]
    alpha, beta = [], []
    v_prev = np.zeros(n)
    b = 0.0
    e0, s = None, None
    resid = np.inf
    for k in range(max_iter):
        w = mv(v)
        a = float(v @ w)
        w = w - a * v - b * v_prev
        if reorth:
            Vm = np.array(V).T
            for _ in range(2):
                w = w - Vm @ (Vm.T @ w)
        alpha.append(a)
        b = float(np.linalg.norm(w))
        e0, s = _lowest(alpha, beta)
        resid = b * abs(s[-1])
        if k + 1 >= min_iter and (resid <= tol * max(1.0, abs(e0)) or b < 1e-14 * max(1.0, abs(e0))):
            break
        if k + 1 == min(max_iter, n):
            break
        beta.append(b)
        v_prev, v = v, w / b
        if keep_vectors:
            V.append(v)
    K = len(alpha)
    if keep_vectors:
        psi = np.array(V[:K]).T @ s
        psi /= np.linalg.norm(psi)
    else:
        psi = None
    return dict(e0=e0, psi0=psi, alpha=np.array(alpha), beta=np.array(beta[:K - 1]),
                iters=K, residual=resid)


def recompute_ground_state(H, phi0, alpha, beta):
    """Eq. change_basis by a second pass: rerun the recurrence with the known
    a_n, b_n and accumulate sum_n s_n |n> without storing the |n>."""
    mv = H if callable(H) else (lambda x: H @ x)
    e0, s = _lowest(alpha, beta)
    v = phi0 / np.linalg.norm(phi0)
    v_prev = np.zeros_like(v)
    psi = s[0] * v
    for k in range(len(alpha) - 1):
        w = mv(v) - alpha[k] * v - (beta[k - 1] if k > 0 else 0.0) * v_prev
        v_prev, v = v, w / beta[k]
        psi = psi + s[k + 1] * v
    return e0, psi / np.linalg.norm(psi)
