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
