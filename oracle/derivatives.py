"""Parameter derivatives of the truncated Hamiltonian and of E0 (gradient
checks for the differentiable solver).

dH~/dt_q is the hop operator of bond q (Eq. hubbard_model: t_q multiplies
sum_s c+_i c_j + h.c.), restricted to the basis like H~ itself; dH~/dU_i is
n_{i up} n_{i dn}; dH~/deps_i is n_{i up} + n_{i dn}.  The Hellmann-Feynman
theorem gives dE0/dtheta = <Omega| dH~/dtheta |Omega> for the normalised,
non-degenerate ground state of H~.

Derivatives of the Green function: ``green_gradient`` takes central finite
differences (step 1e-5) of the oracle's G -- dense ground state of H~(theta)
on the fixed basis, F~+-, and the Lehmann sums over all eigenpairs of H~+-
(``green.green_exact``, which band Lanczos run to exhaustion reproduces; the
band route itself is not differenced, because Krylov directions whose norm
crosses the deflation tolerance as theta moves make its last digits jump) --
for every bond amplitude, U_i and eps_i, and contracts them
with a given output gradient G_bar: Re sum conj(G_bar) dG/dtheta (+ e0_bar
dE0/dtheta).  The basis F~ is held fixed (w_t = 1), as in the definition of
H~ = P H P.

Pins (tests/test_oracle_derivatives.py): central finite differences of the
oracle's own E0 (step 1e-5), which never builds a derivative operator; for G,
the U = 0 closed forms dG/dh = G (dh) G of the one-body resolvent
G = (z - h)^-1 (bond amplitudes and eps_i) and the first-order (Hartree)
term dG_s/dU_i = G E_ii G <n_{i,-s}> at U = 0, and the exact identity
sum_i dG/deps_i = -dG/dz (a uniform orbital-energy shift moves every
excitation energy of G by the same amount) at any U on a sampled basis.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fock
from .green import green_exact
from .hamiltonian import build_csr, hop_terms


def dH_dt(keys, model, q):
    """Hop operator of listed bond q on the basis (CSR)."""
    a, b, _ = model.bonds[q]
    one = model.with_params(bonds=[(a, b, 1.0)])
    r, c, v = hop_terms(keys, one)
    n = len(keys)
    return sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()


def dH_dU(keys, i):
    up, dn = fock.split(keys)
    return sp.diags((fock.bit(up, i) * fock.bit(dn, i)).astype(float))


def dH_deps(keys, i):
    up, dn = fock.split(keys)
    return sp.diags((fock.bit(up, i) + fock.bit(dn, i)).astype(float))


def contract(keys, model, a, b):
    """(d_t, d_U, d_eps) = <a| dH~/dtheta |b> for every bond, U_i, eps_i."""
    dt = np.array([a @ (dH_dt(keys, model, q) @ b) for q in range(len(model.bonds))])
    dU = np.array([a @ (dH_dU(keys, i) @ b) for i in range(model.n_orb)])
    de = np.array([a @ (dH_deps(keys, i) @ b) for i in range(model.n_orb)])
    return dt, dU, de


def central_difference(f, theta, idx, h=1e-5):
    """(f(theta + h e_i) - f(theta - h e_i)) / 2h for each i in idx."""
    out = []
    for i in idx:
        tp = np.array(theta, dtype=float)
        tm = tp.copy()
        tp[i] += h
        tm[i] -= h
        out.append((f(tp) - f(tm)) / (2 * h))
    return np.array(out)


def ground_state_dense(keys, model):
    """(E0, psi0) of H~ on the basis by dense diagonalisation (small bases)."""
    H = build_csr(np.asarray(keys, dtype=np.uint64), model).toarray()
    E, V = np.linalg.eigh(H)
    return E[0], V[:, 0]


def green_selected(keys, model, orbitals, spins, omega, eta=0.0):
    """(E0, G) for a selection mixing spins: G[f, a, b] over the listed
    (orbital, spin) pairs; pairs of different spin do not couple (N_up and
    N_dn are conserved), so each spin runs on its own and the blocks fill in."""
    e0, psi = ground_state_dense(keys, model)
    sel = list(zip(orbitals, spins))
    nf, ns = len(omega), len(sel)
    G = np.zeros((nf, ns, ns), dtype=np.complex128)
    for s in (0, 1):
        idx = [a for a, (_, sp) in enumerate(sel) if sp == s]
        if not idx:
            continue
        Gs = green_exact(keys, model, psi, e0, [sel[a][0] for a in idx], s, omega, eta=eta)
        G[np.ix_(range(nf), idx, idx)] = Gs
    return e0, G


def param_vector(model):
    """theta = (listed bond amplitudes, U_i, eps_i) and its inverse."""
    nb, no = len(model.bonds), model.n_orb
    theta = np.concatenate([[b[2] for b in model.bonds], model.U, model.eps])

    def to_model(th):
        return model.with_params(bonds=[(b[0], b[1], float(v)) for b, v in zip(model.bonds, th[:nb])],
                                 U=th[nb:nb + no], eps=th[nb + no:])

    return theta, to_model


def green_gradient(keys, model, orbitals, spins, omega, G_bar, e0_bar=0.0, eta=0.0, h=1e-5,
                   which=None):
    """(d_t, d_U, d_eps) of L with dL/dG = G_bar (torch convention
    dL/dRe + i dL/dIm) and dL/dE0 = e0_bar, by central differences."""
    theta, to_model = param_vector(model)
    G_bar = np.asarray(G_bar, dtype=np.complex128)

    def loss(th):
        e0, G = green_selected(keys, to_model(th), orbitals, spins, omega, eta)
        return float(np.sum((np.conj(G_bar) * G).real) + e0_bar * e0)

    idx = range(len(theta)) if which is None else which
    g = np.full(len(theta), np.nan)
    g[list(idx)] = central_difference(loss, theta, idx, h)
    nb, no = len(model.bonds), model.n_orb
    return g[:nb], g[nb:nb + no], g[nb + no:]
