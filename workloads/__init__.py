"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *describes* problems: cluster geometry (sites and bonds),
the model parameters (hopping amplitudes, on-site U, orbital energies that
include -mu), the electron sector, the start state of the sampling chain and
seeded random draws (bath parameters, random vectors).  It holds none of the
method's arithmetic: no Hamiltonian, no signs, no Lanczos.  Both the CPU
oracle and the HIP library consume these plain arrays.

Model convention (Hubbard model, Sec. "Model", Eq. hubbard_model, extended by
per-orbital U_i and energies eps_i as the impurity configurations need):

    H = sum_{bonds (i,j,t_ij)} sum_sigma t_ij (c+_{i s} c_{j s} + c+_{j s} c_{i s})
      + sum_i U_i n_{i up} n_{i dn} + sum_{i sigma} eps_i n_{i sigma}

so a nearest-neighbour bond of the paper's "-t sum_ij" carries t_ij = -t, a
next-nearest-neighbour bond t_ij = -t', and eps_i = -mu on a lattice site.
A bond listed twice counts twice (used for period-2 superlattice directions).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import itertools
import math

import numpy as np

__all__ = [
    "Model", "chain", "square", "superlattice", "impurity_plaquette_bath",
    "neel_start", "tiny_impurity", "config_c1", "config_c2", "config_c3", "config_c5",
    "random_vector", "bath_instance_sizes", "matsubara",
]


@dataclass
class Model:
    """A Hubbard-type model on n_orb orbitals in one (N_up, N_dn) sector."""
    n_orb: int
    bonds: list            # list of (i, j, t_ij) with i != j
    U: np.ndarray          # float64[n_orb]
    eps: np.ndarray        # float64[n_orb], includes -mu
    n_up: int
    n_dn: int
    name: str = ""
    coords: list = field(default_factory=list)

    def bond_arrays(self):
        bi = np.array([min(b[0], b[1]) for b in self.bonds], dtype=np.int32)
        bj = np.array([max(b[0], b[1]) for b in self.bonds], dtype=np.int32)
        bt = np.array([b[2] for b in self.bonds], dtype=np.float64)
        return bi, bj, bt

    def with_sector(self, n_up: int, n_dn: int) -> "Model":
        return Model(self.n_orb, list(self.bonds), self.U.copy(), self.eps.copy(),
                     n_up, n_dn, self.name, list(self.coords))

    def with_params(self, bonds=None, U=None, eps=None) -> "Model":
        return Model(self.n_orb, list(self.bonds if bonds is None else bonds),
                     (self.U if U is None else np.asarray(U, np.float64)).copy(),
                     (self.eps if eps is None else np.asarray(eps, np.float64)).copy(),
                     self.n_up, self.n_dn, self.name, list(self.coords))


def _uniform(n, U, mu):
    return np.full(n, float(U)), np.full(n, -float(mu))


def chain(n: int, t: float = 1.0, U: float = 8.0, mu: float = 0.0, pbc: bool = True,
          n_up: int | None = None, n_dn: int | None = None) -> Model:
    """1D cluster of n sites; with pbc the bond (n-1, 0) closes the ring (n > 2)."""
    bonds = [(i, i + 1, -t) for i in range(n - 1)]
    if pbc and n > 2:
        bonds.append((n - 1, 0, -t))
    Uv, ev = _uniform(n, U, mu)
    n_up = n // 2 if n_up is None else n_up
    n_dn = n - n // 2 if n_dn is None else n_dn
    return Model(n, bonds, Uv, ev, n_up, n_dn, f"chain{n}{'p' if pbc else 'o'}",
                 [(i, 0) for i in range(n)])


def square(Lx: int, Ly: int, t: float = 1.0, tp: float = 0.0, U: float = 8.0,
           mu: float = 0.0, pbc: bool = True, n_up=None, n_dn=None) -> Model:
    """Lx x Ly square cluster, site (x, y) -> x + Lx*y.

    NN bonds: +x and +y from every site (wrapped with pbc).  With tp != 0 the
    NNN bonds +x+y and +x-y are added (t_ij = -tp).  No de-duplication: in a
    periodic direction of length 2 the +1 and -1 neighbours coincide and the
    bond appears twice.
    """
    n = Lx * Ly
    idx = lambda x, y: (x % Lx) + Lx * (y % Ly)
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            for dx, dy, amp in ((1, 0, -t), (0, 1, -t)):
                xx, yy = x + dx, y + dy
                if not pbc and (xx >= Lx or yy >= Ly):
                    continue
                bonds.append((idx(x, y), idx(xx, yy), amp))
            if tp != 0.0:
                for dx, dy in ((1, 1), (1, -1)):
                    xx, yy = x + dx, y + dy
                    if not pbc and (xx >= Lx or yy >= Ly or yy < 0):
                        continue
                    bonds.append((idx(x, y), idx(xx, yy), -tp))
    Uv, ev = _uniform(n, U, mu)
    n_up = n // 2 if n_up is None else n_up
    n_dn = n - n // 2 if n_dn is None else n_dn
    coords = [(x, y) for y in range(Ly) for x in range(Lx)]
    return Model(n, bonds, Uv, ev, n_up, n_dn, f"sq{Lx}x{Ly}{'p' if pbc else 'o'}", coords)


def superlattice(R1, R2, t: float = 1.0, U: float = 8.0, mu: float = 0.0,
                 n_up=None, n_dn=None) -> Model:
    """Square-lattice cluster with periodic superlattice vectors R1, R2.

    Sites are the lattice points of the cell spanned by R1, R2 (reduced to a
    canonical representative); each site bonds to its +x and +y neighbours
    reduced modulo the superlattice.
    """
    R = np.array([R1, R2], dtype=np.float64).T            # columns R1, R2
    Rinv = np.linalg.inv(R)
    area = int(round(abs(np.linalg.det(R))))

    def canon(p):
        a = Rinv @ np.array(p, dtype=np.float64)
        fa = np.floor(a + 1e-9)
        q = np.array(p, dtype=np.float64) - R @ fa
        return (int(round(q[0])), int(round(q[1])))

    span = int(max(abs(v) for v in (*R1, *R2))) * 2 + 2
    pts = sorted({canon((x, y)) for x in range(-span, span) for y in range(-span, span)},
                 key=lambda p: (p[1], p[0]))
    assert len(pts) == area, (len(pts), area)
    index = {p: k for k, p in enumerate(pts)}
    bonds = []
    for p in pts:
        for d in ((1, 0), (0, 1)):
            q = canon((p[0] + d[0], p[1] + d[1]))
            bonds.append((index[p], index[q], -t))
    n = area
    Uv, ev = _uniform(n, U, mu)
    n_up = n // 2 if n_up is None else n_up
    n_dn = n - n // 2 if n_dn is None else n_dn
    return Model(n, bonds, Uv, ev, n_up, n_dn, f"super{R1}{R2}", pts)


def impurity_plaquette_bath(seed: int, t: float = 1.0, U: float = 8.0,
                            mu: float | None = None) -> Model:
    """2x2 impurity plaquette (orbitals 0-3) plus 8 bath orbitals (4-11).

    Plaquette: open 2x2, 4 NN bonds.  U and -mu (mu = U/2 by default) act on
    the impurity only.  Bath b (0..7) has energy eps_b ~ U[-2, 2] and couples
    with V_ib ~ U[0.1, 1] to impurity site b mod 4 and to that site's two
    plaquette neighbours (24 hybridisations).  Draw order: the 8 eps_b, then
    the 24 V_ib in (bath, neighbour) order, from numpy's PCG64 at `seed`.
    Half filling: N_up = N_dn = 6.
    """
    mu = U / 2 if mu is None else mu
    rng = np.random.default_rng(seed)
    eps_b = rng.uniform(-2.0, 2.0, size=8)
    V = rng.uniform(0.1, 1.0, size=24)
    plaq = [(0, 1), (1, 3), (3, 2), (2, 0)]
    nbrs = {0: (1, 2), 1: (0, 3), 2: (0, 3), 3: (1, 2)}
    bonds = [(i, j, -t) for i, j in plaq]
    k = 0
    for b in range(8):
        s = b % 4
        for i in (s,) + nbrs[s]:
            bonds.append((i, 4 + b, float(V[k])))
            k += 1
    Uv = np.zeros(12)
    Uv[:4] = U
    ev = np.zeros(12)
    ev[:4] = -mu
    ev[4:] = eps_b
    return Model(12, bonds, Uv, ev, 6, 6, f"imp2x2+8b(seed={seed})")


def neel_start(model: Model) -> int:
    """Start key of the sampling chain: a Neel state (sublattice (x+y) even up).

    Doped sectors drop the highest-index up electron on sublattice A and the
    highest-index down electron on sublattice B until the counts match.
    For an impurity model the plaquette takes the Neel pattern and the baths
    are filled in ascending order of their energy.
    Returns the key (up << 32) | down.
    """
    n = model.n_orb
    if model.coords and len(model.coords) == n:
        A = [i for i in range(n) if (model.coords[i][0] + model.coords[i][1]) % 2 == 0]
        B = [i for i in range(n) if i not in A]
        up, dn = list(A), list(B)
        while len(up) > model.n_up:
            up.remove(max(up))
        while len(dn) > model.n_dn:
            dn.remove(max(dn))
        while len(up) < model.n_up:                       # more up than A holds
            up.append(min(i for i in B if i not in up))
        while len(dn) < model.n_dn:
            dn.append(min(i for i in A if i not in dn))
    else:                                                  # impurity + bath
        imp = [i for i in range(n) if model.U[i] != 0.0]
        bath = sorted((i for i in range(n) if model.U[i] == 0.0), key=lambda i: (model.eps[i], i))
        up = [i for i in imp if i in (0, 3)]
        dn = [i for i in imp if i in (1, 2)]
        fill = bath[: model.n_up - len(up)]
        up += fill
        dn += bath[: model.n_dn - len(dn)]
    ub = sum(1 << i for i in up)
    db = sum(1 << i for i in dn)
    return (ub << 32) | db


# --------------------------------------------------------------------------
# The five benchmark configurations (paper-shaped synthetic clusters)
# --------------------------------------------------------------------------
def config_c1() -> dict:
    """2x4 open cluster, t=1, U=4, mu=0, N_up=N_dn=4 (4900-state sector);
    sampled basis of 2000 states (chain seed 1, burn-in 1e3, <=1e7 steps)."""
    m = square(4, 2, t=1.0, U=4.0, mu=0.0, pbc=False, n_up=4, n_dn=4)
    return dict(model=m, n_f=2000, seed=1, burn_in=1000, max_steps=10**7, beta_s=0.5)


def config_c2() -> dict:
    """4x4 periodic, t=1, t'=-0.3, U=8, mu=0, N_up=N_dn=7; 4M chain states
    (seed 2, burn-in 1e6); Lanczos 200 iterations."""
    m = square(4, 4, t=1.0, tp=-0.3, U=8.0, mu=0.0, pbc=True, n_up=7, n_dn=7)
    # The chain reaches 2.79M distinct states after 1e8 steps; 4M needs 1.66e8,
    # so the step cap is 1e9 and the basis size (the workload) is kept.
    return dict(model=m, n_f=4_000_000, seed=2, burn_in=10**6, max_steps=10**9, beta_s=0.5)


def config_c3(seed: int = 3) -> dict:
    """2x2 plaquette + 8 baths, U=8, half filling; 0.5M chain states."""
    m = impurity_plaquette_bath(seed)
    return dict(model=m, n_f=500_000, seed=seed, burn_in=10**6, max_steps=10**10, beta_s=0.5)


def config_c5() -> dict:
    """4x8 periodic, t=1, t'=-0.3, U=8, mu=0, N_up=N_dn=14; 50M chain states."""
    m = square(8, 4, t=1.0, tp=-0.3, U=8.0, mu=0.0, pbc=True, n_up=14, n_dn=14)
    return dict(model=m, n_f=50_000_000, seed=5, burn_in=10**6, max_steps=10**10, beta_s=0.5)


def tiny_impurity(U: float = 4.0, seed: int = 0, n_up: int = 3, n_dn: int = 3) -> Model:
    """Two interacting sites (bond t = -1, eps = -U/2 +- small offsets that
    lift degeneracies) coupled to four bath orbitals (bath b to site b mod 2,
    V ~ U[0.3, 0.9], eps_b ~ U[-2, 2]); 6 orbitals, small enough for dense
    checks of Green-function derivatives."""
    rng = np.random.default_rng(seed)
    bonds = [(0, 1, -1.0)] + [(b % 2, b, float(rng.uniform(0.3, 0.9))) for b in range(2, 6)]
    Uv = np.array([U, U, 0, 0, 0, 0], dtype=float)
    eps = np.concatenate([[-U / 2 + 0.13, -U / 2 - 0.07], rng.uniform(-2, 2, 4)])
    return Model(6, bonds, Uv, eps, n_up, n_dn, "tiny_impurity", [])


def bath_instance_sizes(n_inst: int = 32, seed: int = 3, lo: int = 100_000,
                        hi: int = 500_000, cap: int = 853_776) -> np.ndarray:
    """Basis sizes of a batch of bath instances, uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed + 1000)
    return np.minimum(rng.integers(lo, hi + 1, size=n_inst), cap)


def random_vector(n: int, seed: int, nvec: int = 1, dtype=np.float64) -> np.ndarray:
    """Seeded U(-1, 1) test vectors, shape (n,) or (n, nvec) row-major."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, nvec) if nvec > 1 else (n,))
    return x.astype(dtype)


def matsubara(n_freq: int, beta_m: float = 50.0) -> np.ndarray:
    """Fermionic Matsubara frequencies omega_n = (2n+1) pi / beta_M, n = 0.."""
    return (2 * np.arange(n_freq) + 1) * math.pi / beta_m
