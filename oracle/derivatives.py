"""Parameter derivatives of the truncated Hamiltonian and of E0 (gradient
checks for the differentiable solver).

dH~/dt_q is the hop operator of bond q (Eq. hubbard_model: t_q multiplies
sum_s c+_i c_j + h.c.), restricted to the basis like H~ itself; dH~/dU_i is
n_{i up} n_{i dn}; dH~/deps_i is n_{i up} + n_{i dn}.  The Hellmann-Feynman
theorem gives dE0/dtheta = <Omega| dH~/dtheta |Omega> for the normalised,
non-degenerate ground state of H~.

Pins (tests/test_oracle_derivatives.py): central finite differences of the
oracle's own E0 (step 1e-5), which never builds a derivative operator.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fock
from .hamiltonian import hop_terms


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
