"""The all-core host product (oracle/spmv.c) equals scipy's product of the
same oracle matrix, on a full sector and on a row slice of a sampled basis
(the form the CPU baseline times)."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import fock, hamiltonian as ham, sampler, spmv


def test_omp_product_equals_scipy():
    m = W.config_c1()["model"]
    keys = fock.sector_keys(8, 4, 4)
    H = ham.build_csr(keys, m)
    x = W.random_vector(len(keys), 4)
    prep = spmv.prepare(H)
    y = spmv.matvec(prep, x)
    assert np.max(np.abs(y - H @ x)) <= 1e-14 * np.max(np.abs(y))
    assert spmv.threads() >= 1


def test_omp_product_on_a_row_slice():
    m = W.impurity_plaquette_bath(3)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 9, 6000, 500, 10**6)
    rows = np.arange(1000, 3000)
    r, c, v = ham.hop_terms_rows(keys, rows, m)
    d = fock.diagonal(keys[rows], m)
    A = sp.coo_matrix((np.concatenate([v, d]), (np.concatenate([r, rows]) - rows[0],
                                               np.concatenate([c, rows]))),
                      shape=(len(rows), len(keys))).tocsr()
    x = W.random_vector(len(keys), 5)
    y = spmv.matvec(spmv.prepare(A), x)
    ref = ham.apply_rows(keys, rows, m, x)
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))
