"""The Hamiltonian restricted to a truncated basis.

``build_csr`` is the definition H~_mn = <x~_m|H|x~_n> (Eq. h_matrix_projected)
written out: every hopping term of Eq. hubbard_model is applied to every basis
state, and a result outside the basis is discarded (App. Lanczos, last
paragraph: discarding is the same as building H~ in the subspace).

Fermion sign of c+_{i s} c_{j s} (i < j) on the same-spin string s, with the
orbital ordering "all up orbitals, then all down orbitals": the Jordan-Wigner
strings of the two operators cancel outside the open interval (i, j), so the
sign is (-1)^(number of s-electrons strictly between i and j).  The other
spin's string never enters.

Pins (tests/test_oracle_hamiltonian.py): the independent Kronecker-product
Jordan-Wigner construction ``jw_full`` below on <= 6-8 orbitals (pattern and
values), H = H^T, the 4-site 36x36 sector of App. BFS vs DFS (off-diagonal
count and values, diagonal multiples of U), and every energy pin of the
Lanczos tests.  The row checker (``hop_terms_rows`` / ``apply_rows``, used for
single rows of bases too large for ``build_csr``) is pinned to the rows of
``build_csr`` and ``offdiag_pattern`` (full sectors and random subsets, one and
several vectors) and to the dense Kronecker matrix; planted mistakes (a sign,
a column, a row, a dropped element) are shown to fail that comparison.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fock


def hop_terms(keys: np.ndarray, model):
    """Off-diagonal elements as COO triples (row m, col n, value).

    For each bond (i, j, t_ij) and spin, each basis state x_n with exactly one
    electron on {i, j} in that spin string is moved to x' = x_n with both bits
    flipped; if x' = x_m is in the basis the element (m, n) gets t_ij * sign.
    """
    keys = np.asarray(keys, dtype=np.uint64)
    up, dn = fock.split(keys)
    rows, cols, vals = [], [], []
    col_all = np.arange(len(keys), dtype=np.int64)
    for (a, b, t) in model.bonds:
        i, j = (a, b) if a < b else (b, a)
        mask = np.uint64((1 << i) | (1 << j))
        between = np.uint64(((1 << j) - 1) & ~((1 << (i + 1)) - 1))
        for shift, s in ((np.uint64(32), up), (np.uint64(0), dn)):
            movable = np.bitwise_count(s & mask) == 1
            if not np.any(movable):
                continue
            src = col_all[movable]
            tgt_key = keys[movable] ^ (mask << shift)
            parity = np.bitwise_count(s[movable] & between) & 1
            sign = 1.0 - 2.0 * parity
            pos = np.searchsorted(keys, tgt_key)
            pos_c = np.minimum(pos, len(keys) - 1)
            found = keys[pos_c] == tgt_key
            rows.append(pos_c[found])
            cols.append(src[found])
            vals.append(t * sign[found])
    if rows:
        return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    z = np.zeros(0, dtype=np.int64)
    return z, z, np.zeros(0)


def hop_terms_rows(keys: np.ndarray, rows: np.ndarray, model):
    """Off-diagonal elements (row m, col n, value) of H~ for the given rows m.

    Same definition as ``hop_terms`` (H~ is symmetric, so the elements of
    row m are the hops applied to x_m), restricted to a subset of rows so
    that single rows of a large basis can be checked.
    """
    keys = np.asarray(keys, dtype=np.uint64)
    rows = np.asarray(rows, dtype=np.int64)
    sub = keys[rows]
    up, dn = fock.split(sub)
    out_r, out_c, out_v = [], [], []
    for (a, b, t) in model.bonds:
        i, j = (a, b) if a < b else (b, a)
        mask = np.uint64((1 << i) | (1 << j))
        between = np.uint64(((1 << j) - 1) & ~((1 << (i + 1)) - 1))
        for shift, s in ((np.uint64(32), up), (np.uint64(0), dn)):
            movable = np.bitwise_count(s & mask) == 1
            tgt = sub[movable] ^ (mask << shift)
            sign = 1.0 - 2.0 * (np.bitwise_count(s[movable] & between) & 1)
            pos = np.minimum(np.searchsorted(keys, tgt), len(keys) - 1)
            found = keys[pos] == tgt
            out_r.append(rows[movable][found])
            out_c.append(pos[found])
            out_v.append(t * sign[found])
    if not out_r:
        z = np.zeros(0, dtype=np.int64)
        return z, z, np.zeros(0)
    return np.concatenate(out_r), np.concatenate(out_c), np.concatenate(out_v)


def apply_rows(keys: np.ndarray, rows: np.ndarray, model, x: np.ndarray) -> np.ndarray:
    """(H~ x)[rows] from the element definition (x of shape (n,) or (n, k))."""
    r, c, v = hop_terms_rows(keys, rows, model)
    d = fock.diagonal(np.asarray(keys, dtype=np.uint64)[rows], model)
    y = d[:, None] * (x[rows] if x.ndim == 2 else x[rows][:, None])
    loc = np.searchsorted(rows, r) if np.all(np.diff(rows) > 0) else None
    assert loc is not None, "rows must be sorted and unique"
    xc = x[c] if x.ndim == 2 else x[c][:, None]
    np.add.at(y, loc, v[:, None] * xc)
    return y if x.ndim == 2 else y[:, 0]


def build_csr(keys: np.ndarray, model) -> sp.csr_matrix:
    """H~ on the basis `keys` (sorted unique) as a float64 CSR matrix."""
    n = len(keys)
    r, c, v = hop_terms(keys, model)
    off = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    off.sum_duplicates()
    d = fock.diagonal(keys, model)
    return (off + sp.diags(d, format="csr")).tocsr()


def offdiag_pattern(keys: np.ndarray, model):
    """Sorted (row, col, value) of the off-diagonal part, duplicates merged."""
    n = len(keys)
    r, c, v = hop_terms(keys, model)
    m = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m = m.tocoo()
    order = np.lexsort((m.col, m.row))
    return m.row[order], m.col[order], m.data[order]


# ---------------------------------------------------------------------------
# Independent pin: second quantisation by Kronecker products (no bit tricks)
# ---------------------------------------------------------------------------
def jw_operators(n_orb: int):
    """Annihilators c_o on 2*n_orb spin-orbitals via the Jordan-Wigner map.

    Spin-orbital o = i for (i, up) and o = n_orb + i for (i, down); the Fock
    index has bit o = occupation of o.  c_o = I (higher) (x) a (x) Z^{(x) o}
    with a = |0><1| and Z = diag(1, -1) on every lower spin-orbital.
    """
    m = 2 * n_orb
    a = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    ops = []
    for o in range(m):
        op = sp.identity(2 ** (m - 1 - o), format="csr")
        op = sp.kron(op, a, format="csr")
        low = sp.identity(1, format="csr")
        for _ in range(o):
            low = sp.kron(low, Z, format="csr")
        op = sp.kron(op, low, format="csr")
        ops.append(op)
    return ops


def jw_full(model) -> sp.csr_matrix:
    """H on the whole 4^n_orb Fock space from Kronecker-product operators."""
    n = model.n_orb
    c = jw_operators(n)
    dim = 4 ** n
    H = sp.csr_matrix((dim, dim))
    for (a, b, t) in model.bonds:
        for s in (0, n):
            ci, cj = c[a + s], c[b + s]
            H = H + t * (ci.T @ cj + cj.T @ ci)
    for i in range(n):
        nu = c[i].T @ c[i]
        nd = c[i + n].T @ c[i + n]
        H = H + model.U[i] * (nu @ nd) + model.eps[i] * (nu + nd)
    return H.tocsr()


def jw_restricted(keys: np.ndarray, model) -> np.ndarray:
    """Dense P H P on `keys`, taken from the Kronecker construction."""
    n = model.n_orb
    up, dn = fock.split(keys)
    idx = (up | (dn << np.uint64(n))).astype(np.int64)
    H = jw_full(model)
    return H[idx][:, idx].toarray()
