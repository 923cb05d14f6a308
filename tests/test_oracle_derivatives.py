"""Pins of the oracle's parameter derivatives: Hellmann-Feynman contractions
against central finite differences of E0 (independent of any derivative
operator)."""
import numpy as np

import workloads as W
from oracle import derivatives as dv, fock, hamiltonian as ham, lanczos as lz, sampler


def _e0(keys, model):
    H = ham.build_csr(keys, model)
    return lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13, max_iter=800)


def test_hellmann_feynman_vs_finite_differences_lattice():
    m = W.square(3, 2, tp=-0.3, U=6.0, mu=1.0, pbc=False, n_up=3, n_dn=2)
    keys = fock.sector_keys(6, 3, 2)
    r = _e0(keys, m)
    dt, dU, de = dv.contract(keys, m, r["psi0"], r["psi0"])
    nb = len(m.bonds)

    def f(theta):
        mm = m.with_params(bonds=[(b[0], b[1], theta[q]) for q, b in enumerate(m.bonds)],
                           U=theta[nb:nb + 6], eps=theta[nb + 6:])
        return _e0(keys, mm)["e0"]

    theta = np.concatenate([[b[2] for b in m.bonds], m.U, m.eps])
    idx = [0, 3, nb - 1, nb + 1, nb + 6, nb + 11]
    fd = dv.central_difference(f, theta, idx)
    hf = np.concatenate([dt, dU, de])[idx]
    assert np.max(np.abs(fd - hf)) < 2e-7


def test_hellmann_feynman_vs_finite_differences_truncated_impurity():
    m = W.impurity_plaquette_bath(4)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 3, 3000, 500, 10**7)
    r = _e0(keys, m)
    dt, dU, de = dv.contract(keys, m, r["psi0"], r["psi0"])
    hyb = [q for q, b in enumerate(m.bonds) if b[1] >= 4]
    for q in hyb[:4]:
        def f(x, q=q):
            bonds = list(m.bonds)
            bonds[q] = (bonds[q][0], bonds[q][1], x[0])
            return _e0(keys, m.with_params(bonds=bonds))["e0"]
        fd = dv.central_difference(f, [m.bonds[q][2]], [0])[0]
        assert abs(fd - dt[q]) < 2e-7
    # bath energy eps_b (orbital 5)
    def fe(x):
        eps = m.eps.copy()
        eps[5] = x[0]
        return _e0(keys, m.with_params(eps=eps))["e0"]
    assert abs(dv.central_difference(fe, [m.eps[5]], [0])[0] - de[5]) < 2e-7
    # bilinear form is symmetric in (a, b) (dH/dtheta is symmetric)
    rng = np.random.default_rng(0)
    a, b = rng.normal(size=len(keys)), rng.normal(size=len(keys))
    x1 = dv.contract(keys, m, a, b)
    x2 = dv.contract(keys, m, b, a)
    for u, v in zip(x1, x2):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Green-function derivatives (central differences of the oracle pipeline)

def _tiny_impurity(U=4.0, seed=0, n_up=3, n_dn=3):
    return W.tiny_impurity(U, seed, n_up, n_dn)


def _one_body(m):
    h = np.diag(m.eps.astype(float))
    for i, j, t in m.bonds:
        h[i, j] += t
        h[j, i] += t
    return h


def test_green_gradient_free_fermion_closed_forms():
    """U = 0, full sector: G = [(z - h)^-1]_sel, so dG/dt_ij = R(E_ij + E_ji)R,
    dG/deps_i = R E_ii R, and to first order in U the self-energy is the
    Hartree term U_i <n_{i,-s}>: dG_s/dU_i = R E_ii R <n_{i,-s}>."""
    m = _tiny_impurity(U=0.0, n_up=3, n_dn=2)
    keys = fock.sector_keys(6, 3, 2)
    sel_o, sel_s = [0, 1, 3], [0, 0, 0]
    omega = W.matsubara(4, 10.0)
    rng = np.random.default_rng(1)
    Gb = rng.normal(size=(4, 3, 3)) + 1j * rng.normal(size=(4, 3, 3))
    d_t, d_U, d_e = dv.green_gradient(keys, m, sel_o, sel_s, omega, Gb)
    h = _one_body(m)
    E, V = np.linalg.eigh(h)
    n_dn = (V[:, :2] ** 2).sum(axis=1)          # <n_{i,dn}> at U = 0
    z = 1j * omega

    def contract(dh):
        tot = 0.0
        for f in range(4):
            R = np.linalg.inv(z[f] * np.eye(6) - h)
            dG = (R @ dh @ R)[np.ix_(sel_o, sel_o)]
            tot += np.sum((np.conj(Gb[f]) * dG).real)
        return tot

    for q, (i, j, _) in enumerate(m.bonds):
        E_ = np.zeros((6, 6))
        E_[i, j] = E_[j, i] = 1.0
        assert abs(d_t[q] - contract(E_)) < 1e-7 * max(1.0, abs(d_t[q]))
    for i in range(6):
        E_ = np.zeros((6, 6))
        E_[i, i] = 1.0
        assert abs(d_e[i] - contract(E_)) < 1e-7 * max(1.0, abs(d_e[i]))
        assert abs(d_U[i] - n_dn[i] * contract(E_)) < 1e-6 * max(1.0, abs(d_U[i]))


def test_green_gradient_uniform_shift_identity_sampled_basis():
    """Shifting every eps_i by d moves H~ by d N on the fixed-N basis and every
    excitation energy of G by d, so sum_i dG/deps_i = -dG/dz at any U, also
    on a sampled basis; dG/dz from differences in the frequency itself."""
    m = _tiny_impurity(U=4.0, seed=2)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 5, 250, 100, 10**6)
    sel_o, sel_s = [0, 1, 2], [0, 0, 1]
    omega = W.matsubara(3, 20.0)
    rng = np.random.default_rng(3)
    Gb = rng.normal(size=(3, 3, 3)) + 1j * rng.normal(size=(3, 3, 3))
    _, _, d_e = dv.green_gradient(keys, m, sel_o, sel_s, omega, Gb)
    hw = 1e-5
    _, Gp = dv.green_selected(keys, m, sel_o, sel_s, omega + hw)
    _, Gm = dv.green_selected(keys, m, sel_o, sel_s, omega - hw)
    dGdz = (Gp - Gm) / (2 * hw) / 1j                # z = i w
    rhs = np.sum((np.conj(Gb) * (-dGdz)).real)
    assert abs(d_e.sum() - rhs) < 1e-6 * max(1.0, abs(rhs))
    # cross-spin entries stay zero (N_up, N_dn conserved)
    _, G = dv.green_selected(keys, m, sel_o, sel_s, omega)
    assert np.all(G[:, 2, :2] == 0) and np.all(G[:, :2, 2] == 0)
