"""Pins of the oracle's Lanczos ground state (App. Lanczos)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fock, hamiltonian as ham, lanczos as lz

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_energies.json")))


def trunc4(x):
    return math.trunc(x * 1e4) / 1e4


def ground(model, keys=None, tol=1e-12, **kw):
    k = fock.sector_keys(model.n_orb, model.n_up, model.n_dn) if keys is None else keys
    H = ham.build_csr(k, model)
    return k, H, lz.lanczos_ground(H, lz.start_vector(k, 11), tol=tol, **kw)


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 8.0, 12.5])
def test_two_site_closed_form(U):
    m = W.chain(2, t=1.0, U=U, mu=0.0, pbc=False, n_up=1, n_dn=1)
    _, _, r = ground(m)
    assert abs(r["e0"] - (U / 2 - math.sqrt(U * U / 4 + 4.0))) < 1e-12


@pytest.mark.parametrize("model", [W.square(4, 2, U=0.0, pbc=False, n_up=4, n_dn=4),
                                   W.chain(6, U=0.0, pbc=True, n_up=3, n_dn=3),
                                   W.square(3, 2, tp=-0.3, U=0.0, pbc=True, n_up=2, n_dn=3)])
def test_free_fermions(model):
    h = np.zeros((model.n_orb, model.n_orb))
    for i, j, t in model.bonds:
        h[i, j] += t
        h[j, i] += t
    e = np.linalg.eigvalsh(h)
    exact = e[: model.n_up].sum() + e[: model.n_dn].sum()
    _, _, r = ground(model)
    assert abs(r["e0"] - exact) < 1e-10


def test_c1_full_sector_dense():
    m = W.config_c1()["model"]
    k, H, r = ground(m)
    w, v = np.linalg.eigh(H.toarray())
    assert abs(r["e0"] - w[0]) < 1e-10 * abs(w[0])
    assert abs(abs(r["psi0"] @ v[:, 0]) - 1.0) < 1e-9
    res = H @ r["psi0"] - r["e0"] * r["psi0"]
    assert np.linalg.norm(res) < 1e-6


def test_second_pass_reconstruction():
    m = W.chain(6, U=4.0, mu=0.0, pbc=True, n_up=3, n_dn=3)
    k, H, r = ground(m, reorth=False, tol=1e-10)
    e0, psi = lz.recompute_ground_state(H, lz.start_vector(k, 11), r["alpha"], r["beta"])
    assert abs(e0 - r["e0"]) < 1e-12
    assert abs(abs(psi @ r["psi0"]) - 1.0) < 1e-10


@pytest.mark.parametrize("n", [4, 8])
def test_paper_table_1d(n):
    m = W.chain(n, t=1.0, U=8.0, mu=4.0, pbc=True)
    _, _, r = ground(m, tol=1e-11)
    assert trunc4(r["e0"] / n) == GOLD["table_1D_energies_f1"][str(n)]


def test_paper_table_2d_small():
    # 2x2 periodic cluster read as the 4-site ring (single bonds)
    m = W.square(2, 2, U=8.0, mu=4.0, pbc=False)
    _, _, r = ground(m)
    assert trunc4(r["e0"] / 4) == GOLD["table_2D_energies_f1"]["2x2"]
    # 2x4 with superlattice ((4,0),(0,2)): the y bonds are doubled
    m = W.square(4, 2, U=8.0, mu=4.0, pbc=True)
    _, _, r = ground(m)
    assert trunc4(r["e0"] / 8) == GOLD["table_2D_energies_f1"]["2x4"]


@pytest.mark.slow
def test_paper_table_12_sites():
    m = W.chain(12, t=1.0, U=8.0, mu=4.0, pbc=True)
    _, _, r = ground(m, tol=1e-9, reorth=False, max_iter=300)
    assert trunc4(r["e0"] / 12) == GOLD["table_1D_energies_f1"]["12"]
    m = W.superlattice((4, 0), (1, 3), U=8.0, mu=4.0)
    _, _, r = ground(m, tol=1e-9, reorth=False, max_iter=300)
    assert trunc4(r["e0"] / 12) == GOLD["table_2D_energies_f1"]["12"]


def test_appendix_afm_states_most_important():
    """|90> = |0101;1010> and |165> (label (up << Nc) | down) carry the largest weight."""
    m = W.chain(4, t=1.0, U=8.0, mu=4.0, pbc=True)
    k, _, r = ground(m)
    up, dn = fock.split(k)
    labels = (up << np.uint64(4)) | dn
    top2 = set(int(x) for x in labels[np.argsort(-r["psi0"] ** 2)[:2]])
    assert top2 == set(GOLD["appendix_graph_4site"]["afm_labels"])


def test_variational_order_nested_bases():
    """Truncation raises the energy (Sec. 1D lattice): E0(B1) >= E0(B2) for B1 in B2."""
    m = W.config_c1()["model"]
    k = fock.sector_keys(8, 4, 4)
    rng = np.random.default_rng(3)
    perm = rng.permutation(len(k))
    last = -np.inf
    for frac in (1.0, 0.6, 0.3, 0.1):
        sub = np.sort(k[perm[: int(frac * len(k))]])
        _, _, r = ground(m, keys=sub)
        assert r["e0"] >= last - 1e-10
        last = r["e0"]


def test_start_vector_is_key_determined():
    k = fock.sector_keys(6, 3, 3)
    v = lz.start_vector(k, 5)
    assert np.all(np.abs(v) <= 1.0)
    sub = k[::3]
    assert np.array_equal(lz.start_vector(sub, 5), v[::3])
    # first splitmix64 output of state 0 (published test value of the generator)
    assert int(lz.splitmix64_first(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_lanczos_without_stored_vectors_same_recurrence():
    """keep_vectors=False keeps the recurrence: the same a_n, b_n and Ritz
    value as the stored form (no reorthogonalisation), and the ground state
    from the second pass of Eq. change_basis."""
    import workloads as W
    from oracle import fock, hamiltonian as ham, lanczos as lz
    m = W.config_c1()["model"]
    keys = fock.sector_keys(8, 4, 4)
    H = ham.build_csr(keys, m)
    v0 = lz.start_vector(keys, 11)
    a = lz.lanczos_ground(H, v0, tol=0.0, max_iter=60, reorth=False)
    b = lz.lanczos_ground(H, v0, tol=0.0, max_iter=60, reorth=False, keep_vectors=False)
    assert b["psi0"] is None
    assert np.array_equal(a["alpha"], b["alpha"]) and np.array_equal(a["beta"], b["beta"])
    assert a["e0"] == b["e0"]
    e0, psi = lz.recompute_ground_state(H, v0, b["alpha"], b["beta"])
    assert abs(abs(psi @ a["psi0"]) - 1.0) < 1e-10
