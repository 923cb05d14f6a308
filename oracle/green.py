"""Green function of the truncated ground state (Sec. Subspace of the Green
function, Sec. Further truncation).

* ``truncate_wt``: normalise |Omega~>, order its coefficients by |c_n|^2 and
  keep the first ones that reach the target weight w_t (Sec. Further
  truncation).  Readings of silent points: ties are broken by ascending key;
  the kept prefix is the shortest whose cumulative weight is >= w_t; the kept
  vector is renormalised (so the spectral sum rule stays exact).
* ``excited_basis``: F~+ = union_mu c+_mu F~ and F~- = union_mu c_mu F~, each
  state kept once (Eq. excited_subspace).  Reading: built per spin sector (the
  paper's f = 1 table sizes are one (N_up+1, N_dn) sector); a block that mixes
  spins is the direct sum of the sector runs.
* ``apply_c``: c+_{i s} or c_{i s} applied to a vector, with the
  Jordan-Wigner sign of the ordering "all up orbitals, then all down":
  (-1)^(number of electrons in orbitals ordered before (i, s)).
* ``green_from_band``: Q = rho^T S from the eigenpairs (E_m, S) of the band
  H_eff (Eq. q_matrix) and the Lehmann sums of Eqs. green_qmatrix, either at
  the real frequencies omega + i eta of the paper (eta > 0; the density of
  states is -Im G_ii / pi) or with omega + i eta replaced by i omega_n
  (Matsubara frequencies, eta = 0).
* ``green_dense``: the definition, Eqs. green_plus / green_minus, by full
  diagonalisation of the N +- 1 Hamiltonians (small systems; used as a pin).
* degenerate ground states (Sec. Subspace of the Green function, last
  sentence): the paper sums G over the degenerate states; the reading used
  here averages them (``degenerate='average'``), which keeps the sum rule and
  the zero-temperature limit; ``'sum'`` gives the literal form.
"""
from __future__ import annotations

import numpy as np

from . import fock
from .band_lanczos import band_lanczos
from .hamiltonian import build_csr


def truncate_wt(keys: np.ndarray, psi: np.ndarray, w_t: float):
    """Keep the most important states up to target weight w_t (sorted keys out)."""
    keys = np.asarray(keys, dtype=np.uint64)
    w = psi ** 2 / float(psi @ psi)
    order = np.lexsort((keys, -w))                    # weight desc, key asc
    cum = np.cumsum(w[order])
    if w_t >= 1.0:
        n_keep = len(keys)
    else:
        n_keep = int(np.searchsorted(cum, w_t, side="left")) + 1
        n_keep = min(n_keep, len(keys))
    kept = np.sort(order[:n_keep])
    k2 = keys[kept]
    p2 = psi[kept]
    return k2, p2 / np.linalg.norm(p2)


def _jw_sign(up, dn, i, spin):
    below = np.uint64((1 << i) - 1)
    if spin == 0:
        par = np.bitwise_count(up & below)
    else:
        par = np.bitwise_count(up) + np.bitwise_count(dn & below)
    return 1.0 - 2.0 * (par & 1)


def _image(keys, i, spin, create):
    up, dn = fock.split(keys)
    s = up if spin == 0 else dn
    b = np.uint64(1 << i)
    ok = (s & b) == 0 if create else (s & b) != 0
    shift = np.uint64(32) if spin == 0 else np.uint64(0)
    tgt = keys[ok] ^ (b << shift)
    sign = _jw_sign(up[ok], dn[ok], i, spin)
    return ok, tgt, sign


def excited_basis(keys: np.ndarray, orbitals, spin: int, create: bool) -> np.ndarray:
    """Sorted-unique images of the basis under c+_{i spin} (or c_{i spin})."""
    keys = np.asarray(keys, dtype=np.uint64)
    parts = [_image(keys, i, spin, create)[1] for i in orbitals]
    return np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.uint64)


def apply_c(keys, psi, keys_out, i, spin, create):
    """c+_{i spin}|psi> (create) or c_{i spin}|psi> expressed on keys_out."""
    keys = np.asarray(keys, dtype=np.uint64)
    ok, tgt, sign = _image(keys, i, spin, create)
    out = np.zeros(len(keys_out))
    pos = np.searchsorted(keys_out, tgt)
    assert np.all(keys_out[np.minimum(pos, len(keys_out) - 1)] == tgt)
    out[pos] = sign * psi[ok]
    return out


def lehmann_from_band(T, rho):
    """Eigenpairs of H_eff and Q = rho^T S (Eq. q_matrix)."""
    E, S = np.linalg.eigh(T)
    Q = rho.T @ S
    return E, Q


def green_sum(E, Q, e0, z, particle: bool):
    """G+(z) = sum_m Q_mu m Q_nu m / (z + e0 - E_m); G-(z) = ... /(z - e0 + E_m)."""
    z = np.asarray(z)
    den = (z[:, None] + e0 - E[None, :]) if particle else (z[:, None] - e0 + E[None, :])
    return np.einsum("am,bm,fm->fab", Q, Q, 1.0 / den)


def green_from_band(H_plus, B_plus, H_minus, B_minus, e0, omega, max_dim=None):
    """G(i omega_n) = G+ + G- for one spin sector from two band runs."""
    z = 1j * np.asarray(omega)
    out = 0.0
    for H, B, part in ((H_plus, B_plus, True), (H_minus, B_minus, False)):
        r = band_lanczos(H, B, max_dim=max_dim)
        E, Q = lehmann_from_band(r["T"], r["rho"])
        out = out + green_sum(E, Q, e0, z, part)
    return out


def frequency_argument(omega, eta: float = 0.0):
    """z of the Lehmann sums: i omega_n (eta == 0) or omega + i eta (eta > 0)."""
    omega = np.asarray(omega, dtype=np.float64)
    return omega + 1j * eta if eta > 0 else 1j * omega


def green_mcd(keys, model, psi0, e0, orbitals, spin, omega, max_dim=None,
              w_t: float = 1.0, return_parts=False, eta: float = 0.0):
    """Full MCD Green-function pipeline for one spin (Sec. GreenFunction).

    w_t truncation of |Omega~> -> F~+ and F~- -> start blocks c+|Omega~>,
    c|Omega~> -> band Lanczos on H~+ and H~- -> Q -> G(i omega_n).
    """
    k_t, p_t = truncate_wt(keys, psi0, w_t)
    up_shift = 1 if spin == 0 else 0
    res = {}
    for create in (True, False):
        d = 1 if create else -1
        m2 = model.with_sector(model.n_up + d * up_shift, model.n_dn + d * (1 - up_shift))
        kx = excited_basis(k_t, orbitals, spin, create)
        Hx = build_csr(kx, m2)
        B = np.stack([apply_c(k_t, p_t, kx, i, spin, create) for i in orbitals], axis=1)
        r = band_lanczos(Hx, B, max_dim=max_dim)
        E, Q = lehmann_from_band(r["T"], r["rho"])
        res[create] = (E, Q, kx, r["K"])
    z = frequency_argument(omega, eta)
    Gp = green_sum(res[True][0], res[True][1], e0, z, True)
    Gm = green_sum(res[False][0], res[False][1], e0, z, False)
    if return_parts:
        return Gp + Gm, dict(plus=res[True], minus=res[False], keys_t=k_t, psi_t=p_t)
    return Gp + Gm


def green_exact(keys, model, psi0, e0, orbitals, spin, omega, eta: float = 0.0):
    """What band Lanczos run to exhaustion computes, written out: the Lehmann
    sums of Eqs. green_qmatrix over every eigenpair of H~+ and H~- on F~+ and
    F~- (dense; no target-weight cut), start vectors c+|psi0> and c|psi0>."""
    keys = np.asarray(keys, dtype=np.uint64)
    z = frequency_argument(omega, eta)
    up_shift = 1 if spin == 0 else 0
    G = 0.0
    for create in (True, False):
        d = 1 if create else -1
        m2 = model.with_sector(model.n_up + d * up_shift, model.n_dn + d * (1 - up_shift))
        kx = excited_basis(keys, orbitals, spin, create)
        if len(kx) == 0:
            continue
        E, S = np.linalg.eigh(build_csr(kx, m2).toarray())
        B = np.stack([apply_c(keys, psi0, kx, i, spin, create) for i in orbitals], axis=1)
        G = G + green_sum(E, B.T @ S, e0, z, create)
    return G


def green_dense(model, gs_keys, gs_vecs, e0, orbitals, spin, z, degenerate="average"):
    """Eqs. green_plus / green_minus summed over eigenstates of full sectors.

    gs_vecs: (N, d) degenerate ground states on gs_keys (sorted full sector).
    """
    d = gs_vecs.shape[1]
    up_shift = 1 if spin == 0 else 0
    G = 0.0
    for create in (True, False):
        dd = 1 if create else -1
        m2 = model.with_sector(model.n_up + dd * up_shift, model.n_dn + dd * (1 - up_shift))
        if not (0 <= m2.n_up <= model.n_orb and 0 <= m2.n_dn <= model.n_orb):
            continue
        kx = fock.sector_keys(model.n_orb, m2.n_up, m2.n_dn)
        Hx = build_csr(kx, m2).toarray()
        E, S = np.linalg.eigh(Hx)
        for g in range(d):
            B = np.stack([apply_c(gs_keys, gs_vecs[:, g], kx, i, spin, create)
                          for i in orbitals], axis=1)
            Q = B.T @ S                  # <E_m| c+_nu |Omega> (real)
            G = G + green_sum(E, Q, e0, z, create)
    return G / d if degenerate == "average" else G
