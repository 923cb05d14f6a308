"""Band Lanczos for several start vectors (App. Band Lanczos).

The paper cites the band Lanczos method of the Templates book (Bai et al.
2000, Freund's section) without restating it.  This is that algorithm for a
real symmetric operator, written from its description:

* candidates v^_1..v^_p start as the start vectors b_1..b_p; p_c is the
  current block width; I is the set of indices whose candidates were
  deflated while a later vector still couples to them;
* each step j: deflate v^_j if ||v^_j|| <= dtol (shrinking p_c and shifting
  the later candidates down); otherwise normalise it into v_j, orthogonalise
  the p_c - 1 pending candidates against v_j, form the new candidate
  A v_j and orthogonalise it against the band v_{j-p_c}..v_{j-1} and against
  v_k for k in I and k = j, recording every coefficient in T (or, for the
  coefficients that refer to a start vector, in rho, so B = V rho).

The oracle adds full reorthogonalisation of each new candidate against all
accepted vectors (two classical Gram-Schmidt passes; coefficients dropped).
Deflation tolerance (reading of a silent point): dtol = 1e-10 times the
largest start-vector norm.

The result spans the block Krylov space K_r^L of the paper; T is the
projected (banded) H_eff, rho the start block in the Lanczos basis.

Pins: tests/test_oracle_green.py checks that p = 1 reproduces scalar
Lanczos, that the run exhausts to the exact eigenvalues on small spaces, that
rho reproduces B, and the Green functions built from it against dense
Lehmann sums and closed forms.
"""
from __future__ import annotations

import numpy as np


def band_lanczos(H, B: np.ndarray, max_dim: int | None = None, dtol_rel: float = 1e-10,
                 reorth: bool = True):
    """Returns dict(T (K x K), rho (K x p), V (N x K), K)."""
    mv = H if callable(H) else (lambda x: H @ x)
    N, p = B.shape
    max_dim = N if max_dim is None else min(max_dim, N)
    dtol = dtol_rel * max(np.linalg.norm(B[:, k]) for k in range(p))
    vhat = {k + 1: B[:, k].astype(np.float64).copy() for k in range(p)}   # 1-based slots
    Vs = np.zeros((N, max_dim))       # column j-1 holds v_j
    V = {}
    t = {}            # (i, k) -> value for k >= 1
    rho = {}          # (i, m) -> value, m = start-vector column (1-based)
    I = []
    pc = p
    j = 0
    while True:
        j += 1
        # (1) deflation test
        while True:
            nrm = np.linalg.norm(vhat[j])
            if nrm > dtol:
                break
            if j - pc > 0:
                I.append(j - pc)
            pc -= 1
            if pc == 0:
                break
            for k in range(j, j + pc):
                vhat[k] = vhat[k + 1]
            del vhat[j + pc]
        if pc == 0:
            j -= 1
            break
        # (2) normalise
        src = j - pc
        if src > 0:
            t[(j, src)] = nrm
        else:
            rho[(j, src + p)] = nrm
        Vs[:, j - 1] = vhat.pop(j) / nrm
        V[j] = Vs[:, j - 1]
        # (3) pending candidates against v_j
        for k in range(j + 1, j + pc):
            c = float(V[j] @ vhat[k])
            src = k - pc
            if src > 0:
                t[(j, src)] = c
            else:
                rho[(j, src + p)] = c
            vhat[k] = vhat[k] - c * V[j]
        # (4) new candidate
        w = mv(V[j])
        # (5) band part, using the transposed entries already known
        for k in range(max(1, j - pc), j):
            c = t.get((j, k), 0.0)
            t[(k, j)] = c
            w = w - c * V[k]
        # (6) deflated indices and j itself
        for k in sorted(set(I) | {j}):
            c = float(V[k] @ w)
            t[(k, j)] = c
            w = w - c * V[k]
        # (7)
        for k in I:
            t[(j, k)] = t[(k, j)]
        if reorth:
            Vm = Vs[:, :j]
            for _ in range(2):
                w = w - Vm @ (Vm.T @ w)
        vhat[j + pc] = w
        if j >= max_dim:
            break
    K = j
    T = np.zeros((K, K))
    for (a, b), v in t.items():
        if a <= K and b <= K:
            T[a - 1, b - 1] = v
    R = np.zeros((K, p))
    for (a, m), v in rho.items():
        if a <= K:
            R[a - 1, m - 1] = v
    return dict(T=T, rho=R, V=Vs[:, :K], K=K)
