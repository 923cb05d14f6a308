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
