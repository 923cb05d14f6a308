"""Pins of the oracle's basis and Hamiltonian construction.

The vectorised bit-twiddling builder (oracle.hamiltonian.build_csr) is checked
against an independent Kronecker-product Jordan-Wigner construction, against
the 36-state 4-site sector of the paper's appendix (BFS vs DFS), and against
the binomial sector sizes the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fock, hamiltonian as ham

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_energies.json")))


def test_sector_sizes():
    assert fock.sector_size(4, 2, 2) == GOLD["appendix_graph_4site"]["sector_size"]
    assert len(fock.sector_keys(4, 2, 2)) == 36
    assert fock.sector_size(16, 8, 8) == GOLD["table_reduce_green_f1_wt1"]["F_size"]
    # the excited space at f = 1 is one spin sector: (9, 8)
    assert fock.sector_size(16, 9, 8) == GOLD["table_reduce_green_f1_wt1"]["Fpm_size"]
    assert round(0.05 * fock.sector_size(16, 8, 8)) == GOLD["N_f_16site_f005"]
    for n, a, b in ((8, 4, 4), (6, 2, 3), (12, 6, 6)):
        k = fock.sector_keys(n, a, b)
        assert len(k) == math.comb(n, a) * math.comb(n, b)
        assert np.all(k[1:] > k[:-1])


MODELS = [
    W.chain(2, U=4.0, pbc=False, n_up=1, n_dn=1),
    W.chain(4, U=8.0, mu=4.0, pbc=True),
    W.chain(5, U=3.0, mu=1.0, pbc=True, n_up=2, n_dn=3),
    W.square(4, 2, U=4.0, pbc=False, n_up=4, n_dn=4),
    W.square(3, 2, tp=-0.3, U=8.0, pbc=True, n_up=3, n_dn=2),
    W.square(2, 2, U=8.0, pbc=True),                 # doubled bonds (period 2)
]


def _random_model(seed, n=6):
    rng = np.random.default_rng(seed)
    bonds = [(int(i), int(j), float(rng.normal())) for i in range(n) for j in range(i + 1, n)
             if rng.uniform() < 0.6]
    return W.Model(n, bonds, rng.uniform(0, 8, n), rng.uniform(-2, 2, n), 3, 2, "rand")


@pytest.mark.parametrize("model", MODELS + [_random_model(s) for s in range(3)])
def test_csr_equals_jordan_wigner_full_sector(model):
    k = fock.sector_keys(model.n_orb, model.n_up, model.n_dn)
    H = ham.build_csr(k, model).toarray()
    Hj = ham.jw_restricted(k, model)
    assert np.array_equal(H, Hj)
    assert np.array_equal(H, H.T)


@pytest.mark.parametrize("seed", range(4))
def test_csr_equals_jordan_wigner_truncated(seed):
    """P H P on a random subset: out-of-basis images are discarded."""
    model = _random_model(100 + seed)
    k = fock.sector_keys(model.n_orb, model.n_up, model.n_dn)
    rng = np.random.default_rng(seed)
    sub = np.sort(rng.choice(k, size=len(k) // 3, replace=False))
    H = ham.build_csr(sub, model).toarray()
    assert np.array_equal(H, ham.jw_restricted(sub, model))


def test_appendix_4site_matrix():
    """36x36 sector; open chain off-diagonals are all -t = -1, diagonal U*n_U."""
    g = GOLD["appendix_graph_4site"]
    k = fock.sector_keys(4, 2, 2)
    H = ham.build_csr(k, W.chain(4, U=g["U"], mu=0.0, pbc=False)).toarray()
    off = H - np.diag(np.diag(H))
    assert set(off[off != 0]) == {g["offdiag_value"]}
    assert (off != 0).sum() == 144
    assert set(np.diag(H)) == {0.0, 8.0, 16.0}
    Hr = ham.build_csr(k, W.chain(4, U=8.0, mu=0.0, pbc=True)).toarray()
    offr = Hr - np.diag(np.diag(Hr))
    assert (offr != 0).sum() == 192 and set(offr[offr != 0]) == {-1.0, 1.0}


def test_conservation_and_hermiticity_random_basis():
    m = W.square(4, 4, tp=-0.3, U=8.0, pbc=True, n_up=7, n_dn=7)
    rng = np.random.default_rng(5)
    ups = fock.strings(16, 7)
    keys = np.unique((rng.choice(ups, 3000) << np.uint64(32)) | rng.choice(ups, 3000))
    r, c, v = ham.hop_terms(keys, m)
    ku, kd = fock.split(keys[r])
    assert np.all(np.bitwise_count(ku) == 7) and np.all(np.bitwise_count(kd) == 7)
    H = ham.build_csr(keys, m)
    assert abs(H - H.T).max() == 0.0
    # each image differs from its source in exactly two bits of one spin string
    x = keys[r] ^ keys[c]
    assert np.all(np.bitwise_count(x) == 2)


# --- the row checker used at full size (hop_terms_rows / apply_rows) --------
# The full-size parity tests and the CPU baseline check single rows of H~ x
# with oracle.hamiltonian.apply_rows; these tests tie it to the whole-matrix
# definition (build_csr, itself pinned to the Kronecker construction above)
# and to the dense Kronecker matrix directly.
def _row_cases():
    out = []
    for model in MODELS[1:] + [_random_model(7)]:
        k = fock.sector_keys(model.n_orb, model.n_up, model.n_dn)
        out.append((model, k))
        rng = np.random.default_rng(model.n_orb)
        out.append((model, np.sort(rng.choice(k, size=max(2, len(k) // 3), replace=False))))
    return out


@pytest.mark.parametrize("case", range(len(MODELS[1:]) * 2 + 2))
def test_apply_rows_equals_matrix_rows(case):
    model, keys = _row_cases()[case]
    H = ham.build_csr(keys, model)
    rng = np.random.default_rng(case)
    n = len(keys)
    rows = np.sort(rng.choice(n, size=max(1, n // 4), replace=False))
    x1 = rng.uniform(-1, 1, n)
    x2 = rng.uniform(-1, 1, (n, 3))
    y1 = ham.apply_rows(keys, rows, model, x1)
    y2 = ham.apply_rows(keys, rows, model, x2)
    assert y1.shape == (len(rows),) and y2.shape == (len(rows), 3)
    assert np.max(np.abs(y1 - (H @ x1)[rows])) <= 1e-15 * max(1.0, np.max(np.abs(y1)))
    assert np.max(np.abs(y2 - (H @ x2)[rows])) <= 1e-15 * max(1.0, np.max(np.abs(y2)))
    # every row at once, against the dense Kronecker-product matrix
    if n <= 1000:
        Hj = ham.jw_restricted(keys, model)
        yall = ham.apply_rows(keys, np.arange(n), model, x1)
        assert np.max(np.abs(yall - Hj @ x1)) <= 1e-13


@pytest.mark.parametrize("case", range(len(MODELS[1:]) * 2 + 2))
def test_hop_terms_rows_equal_pattern_rows(case):
    model, keys = _row_cases()[case]
    pr, pc, pv = ham.offdiag_pattern(keys, model)
    rng = np.random.default_rng(100 + case)
    rows = np.sort(rng.choice(len(keys), size=max(1, len(keys) // 5), replace=False))
    r, c, v = ham.hop_terms_rows(keys, rows, model)
    # merge duplicates (a pair listed twice) the way the pattern does
    import scipy.sparse as sp
    m = sp.coo_matrix((v, (r, c)), shape=(len(keys), len(keys))).tocsr()
    m.sum_duplicates()
    m = m.tocoo()
    o = np.lexsort((m.col, m.row))
    sel = np.isin(pr, rows)
    assert np.array_equal(m.row[o], pr[sel]) and np.array_equal(m.col[o], pc[sel])
    assert np.array_equal(m.data[o], pv[sel])


def _planted(kind, keys, rows, model, x):
    """apply_rows with one plausible mistake planted in its element list."""
    r, c, v = ham.hop_terms_rows(keys, rows, model)
    if kind == "sign":          # one element with the wrong fermion sign
        v = v.copy()
        v[len(v) // 2] = -v[len(v) // 2]
    elif kind == "column":      # one element read from the neighbouring column
        c = c.copy()
        c[len(c) // 2] = (c[len(c) // 2] + 1) % len(keys)
    elif kind == "row":         # one element credited to the neighbouring row
        r = r.copy()
        i = len(r) // 2
        r[i] = rows[(np.searchsorted(rows, r[i]) + 1) % len(rows)]
    elif kind == "dropped":     # one element missing
        r, c, v = np.delete(r, len(r) // 2), np.delete(c, len(c) // 2), np.delete(v, len(v) // 2)
    d = fock.diagonal(np.asarray(keys, dtype=np.uint64)[rows], model)
    y = d * x[rows]
    np.add.at(y, np.searchsorted(rows, r), v * x[c])
    return y


@pytest.mark.parametrize("kind", ["sign", "column", "row", "dropped"])
def test_row_pin_catches_planted_mistakes(kind):
    """The comparison above fails for each planted mistake (so it is a pin)."""
    model, keys = _row_cases()[1]
    H = ham.build_csr(keys, model)
    rng = np.random.default_rng(0)
    rows = np.arange(0, len(keys), 2)
    x = rng.uniform(-1, 1, len(keys))
    good = _planted("none", keys, rows, model, x)
    assert np.max(np.abs(good - (H @ x)[rows])) <= 1e-15 * np.max(np.abs(good))
    bad = _planted(kind, keys, rows, model, x)
    assert np.max(np.abs(bad - (H @ x)[rows])) > 1e-6
