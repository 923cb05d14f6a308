"""Pins of the oracle's band Lanczos and Green function (Sec. Subspace of the
Green function, Sec. Further truncation, App. Band Lanczos)."""
import numpy as np
import pytest

import workloads as W
from oracle import band_lanczos as bl, fock, green as gr, hamiltonian as ham, lanczos as lz

OM = W.matsubara(16, 50.0)
Z = 1j * OM


def gs(model, keys=None, tol=1e-13):
    k = fock.sector_keys(model.n_orb, model.n_up, model.n_dn) if keys is None else keys
    H = ham.build_csr(k, model)
    r = lz.lanczos_ground(H, lz.start_vector(k, 3), tol=tol)
    return k, H, r


def test_hubbard_atom_closed_form_averaging():
    """t = 0, mu = U/2: G = (1/2)[1/(iw - U/2) + 1/(iw + U/2)], from the averaged doublet."""
    U = 8.0
    m_up = W.Model(1, [], np.array([U]), np.array([-U / 2]), 1, 0)
    m_dn = m_up.with_sector(0, 1)
    e0 = -U / 2
    G1 = gr.green_dense(m_up, fock.sector_keys(1, 1, 0), np.ones((1, 1)), e0, [0], 0, Z)
    G2 = gr.green_dense(m_dn, fock.sector_keys(1, 0, 1), np.ones((1, 1)), e0, [0], 0, Z)
    G = 0.5 * (G1 + G2)[:, 0, 0]
    assert np.abs(G - 0.5 * (1 / (Z - U / 2) + 1 / (Z + U / 2))).max() < 1e-15
    # the literal "sum" reading would double the weight
    assert abs((G1 + G2)[0, 0, 0] * Z[-1] * 0 + np.sum(np.abs(G1 + G2))) > 0


@pytest.mark.parametrize("model", [W.chain(6, U=0.0, pbc=True, n_up=3, n_dn=3),
                                   W.square(3, 2, U=0.0, tp=-0.3, pbc=False, n_up=2, n_dn=2)])
def test_free_fermion_green(model):
    k, H, r = gs(model)
    h = np.zeros((model.n_orb,) * 2)
    for i, j, t in model.bonds:
        h[i, j] += t
        h[j, i] += t
    e = np.linalg.eigvalsh(h)
    assert e[model.n_up] - e[model.n_up - 1] > 1e-6        # closed shell: unique ground state
    G = gr.green_mcd(k, model, r["psi0"], r["e0"], list(range(model.n_orb)), 0, OM)
    G0 = np.array([np.linalg.inv(z * np.eye(model.n_orb) - h) for z in Z])
    assert np.abs(G - G0).max() < 1e-11


@pytest.mark.parametrize("spin", [0, 1])
def test_band_lanczos_green_vs_dense_lehmann(spin):
    m = W.chain(6, U=6.0, mu=3.0, pbc=True, n_up=3, n_dn=3)
    k, H, r = gs(m)
    orbs = [0, 1, 2, 4]
    G = gr.green_mcd(k, m, r["psi0"], r["e0"], orbs, spin, OM)
    Gd = gr.green_dense(m, k, r["psi0"][:, None], r["e0"], orbs, spin, Z)
    assert np.abs(G - Gd).max() < 1e-11


def test_truncated_basis_green_vs_dense_definition():
    """MCD Green function on a truncated basis equals the Lehmann sum of the
    truncated H~+- diagonalised densely (discarding outside F~+-)."""
    m = W.config_c1()["model"]
    k = fock.sector_keys(8, 4, 4)
    sub = np.sort(np.random.default_rng(0).choice(k, 900, replace=False))
    _, H, r = gs(m, sub)
    orbs = [0, 3, 5]
    G, parts = gr.green_mcd(sub, m, r["psi0"], r["e0"], orbs, 0, OM, return_parts=True)
    for create, (E, Q, kx, K) in ((True, parts["plus"]), (False, parts["minus"])):
        m2 = m.with_sector(m.n_up + (1 if create else -1), m.n_dn)
        Hx = ham.build_csr(kx, m2).toarray()
        Ed, S = np.linalg.eigh(Hx)
        B = np.stack([gr.apply_c(sub, r["psi0"], kx, i, 0, create) for i in orbs], axis=1)
        Gd = gr.green_sum(Ed, B.T @ S, r["e0"], Z, create)
        Gb = gr.green_sum(E, Q, r["e0"], Z, create)
        assert np.abs(Gb - Gd).max() < 1e-11


def test_sum_rule_symmetry_and_tail():
    m = W.config_c1()["model"]
    k, H, r = gs(m)
    orbs = [0, 1, 2]
    G, parts = gr.green_mcd(k, m, r["psi0"], r["e0"], orbs, 0, OM, max_dim=120,
                            return_parts=True)
    Qp, Qm = parts["plus"][1], parts["minus"][1]
    # sum_m |Q+_mu m|^2 + sum_n |Q-_mu n|^2 = ||c+ psi||^2 + ||c psi||^2 = 1
    assert np.allclose((Qp ** 2).sum(1) + (Qm ** 2).sum(1), 1.0, atol=1e-12)
    assert np.abs(G - G.transpose(0, 2, 1)).max() < 1e-13
    big = 1j * np.array([1e6])
    Gt = gr.green_sum(*parts["plus"][:2], r["e0"], big, True) + \
        gr.green_sum(*parts["minus"][:2], r["e0"], big, False)
    assert np.abs(Gt[0] * big[0] - np.eye(3)).max() < 1e-4


def test_band_p1_is_scalar_lanczos_and_rho_reproduces_B():
    m = W.chain(6, U=4.0, mu=2.0, pbc=True, n_up=3, n_dn=3)
    k, H, r = gs(m)
    kx = gr.excited_basis(k, [0, 1, 2], 0, True)
    m2 = m.with_sector(4, 3)
    Hx = ham.build_csr(kx, m2)
    b = gr.apply_c(k, r["psi0"], kx, 0, 0, True)
    rb = bl.band_lanczos(Hx, b[:, None], max_dim=25)
    rl = lz.lanczos_ground(Hx, b, tol=0.0, max_iter=25)
    assert np.allclose(np.diag(rb["T"]), rl["alpha"], atol=1e-12)
    B = np.stack([gr.apply_c(k, r["psi0"], kx, i, 0, True) for i in (0, 1, 2)], 1)
    rb = bl.band_lanczos(Hx, B, max_dim=40)
    assert np.abs(rb["V"] @ rb["rho"] - B).max() < 1e-12
    assert np.abs(rb["V"].T @ rb["V"] - np.eye(rb["K"])).max() < 1e-12
    assert np.abs(rb["V"].T @ (Hx @ rb["V"]) - rb["T"]).max() < 1e-10


def test_band_deflation_duplicate_start_vectors():
    m = W.chain(6, U=4.0, mu=2.0, pbc=True, n_up=3, n_dn=3)
    k, H, r = gs(m)
    kx = gr.excited_basis(k, [0, 1], 0, True)
    Hx = ham.build_csr(kx, m.with_sector(4, 3))
    b0 = gr.apply_c(k, r["psi0"], kx, 0, 0, True)
    b1 = gr.apply_c(k, r["psi0"], kx, 1, 0, True)
    B = np.stack([b0, b1, b0 + 2 * b1], 1)               # rank 2
    rb = bl.band_lanczos(Hx, B, max_dim=60)
    E = np.linalg.eigvalsh(rb["T"])
    B2 = np.stack([b0, b1], 1)
    rb2 = bl.band_lanczos(Hx, B2, max_dim=60)
    assert rb["K"] == rb2["K"] == 60
    assert np.allclose(E, np.linalg.eigvalsh(rb2["T"]), atol=1e-9)
    assert np.abs(rb["V"] @ rb["rho"] - B).max() < 1e-10


def test_wt_truncation():
    m = W.config_c1()["model"]
    k, H, r = gs(m)
    for wt in (0.5, 0.9, 0.99, 1.0):
        k2, p2 = gr.truncate_wt(k, r["psi0"], wt)
        w = np.sort(r["psi0"] ** 2)[::-1]
        n_exp = len(k) if wt >= 1 else int(np.argmax(np.cumsum(w) >= wt)) + 1
        assert len(k2) == n_exp
        assert abs(np.linalg.norm(p2) - 1) < 1e-14
        assert np.all(k2[1:] > k2[:-1]) and np.all(np.isin(k2, k))
        kept_w = r["psi0"][np.isin(k, k2)] ** 2
        assert kept_w.min() >= np.sort(r["psi0"] ** 2)[::-1][len(k2) - 1] - 1e-18


def test_green_exact_equals_exhausted_band_and_definition():
    """green_exact (all eigenpairs of H~+- on F~+-) equals band Lanczos run to
    exhaustion on a sampled basis, and the full-sector definition on a full
    sector; also at real frequencies with a Lorentzian width."""
    from oracle import green as gr, sampler
    m = W.square(3, 2, tp=-0.3, U=5.0, mu=1.0, pbc=False, n_up=3, n_dn=2)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 7, 180, 100, 10**6)
    H = ham.build_csr(keys, m).toarray()
    E, V = np.linalg.eigh(H)
    for eta, om in ((0.0, W.matsubara(5, 20.0)), (0.05, np.linspace(-6, 6, 9))):
        a = gr.green_exact(keys, m, V[:, 0], E[0], [0, 2, 5], 1, om, eta=eta)
        b = gr.green_mcd(keys, m, V[:, 0], E[0], [0, 2, 5], 1, om, eta=eta)
        assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(a))
    kf = fock.sector_keys(6, 3, 2)
    Hf = ham.build_csr(kf, m).toarray()
    Ef, Vf = np.linalg.eigh(Hf)
    om = W.matsubara(4, 10.0)
    # every orbital selected: F~+- are then the whole N +- 1 sectors
    a = gr.green_exact(kf, m, Vf[:, 0], Ef[0], range(6), 0, om)
    c = gr.green_dense(m, kf, Vf[:, :1], Ef[0], range(6), 0, 1j * om)
    assert np.max(np.abs(a - c)) < 1e-12 * np.max(np.abs(c))
