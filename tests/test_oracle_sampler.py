"""Pins of the oracle's basis sampler (Sec. Subspace of the ground state;
variant-1 acceptance with a single random hop, Sec. Other sampling methods)."""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import fock, hamiltonian as ham, sampler


def test_c_and_python_chains_agree_bit_for_bit():
    c = W.config_c1()
    m = c["model"]
    a, sa = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"], c["max_steps"])
    b, sb = sampler.chain_python(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                 c["max_steps"])
    assert sa == sb and np.array_equal(a, b) and len(a) == c["n_f"]
    fock.check_sector(a, m)


def test_impurity_chain_agrees():
    m = W.impurity_plaquette_bath(7)
    st = W.neel_start(m)
    a, sa = sampler.chain_c(m, st, 9, 3000, 500, 10**6)
    b, sb = sampler.chain_python(m, st, 9, 3000, 500, 10**6)
    assert sa == sb and np.array_equal(a, b)
    fock.check_sector(a, m)


def test_neel_start_states():
    m = W.config_c1()["model"]
    k = W.neel_start(m)
    up, dn = k >> 32, k & 0xFFFFFFFF
    assert bin(up).count("1") == 4 and bin(dn).count("1") == 4 and up & dn == 0
    m2 = W.config_c2()["model"]
    k2 = W.neel_start(m2)
    assert bin(k2 >> 32).count("1") == 7 and bin(k2 & 0xFFFFFFFF).count("1") == 7


@pytest.mark.parametrize("model", [W.chain(4, U=8.0, mu=4.0, pbc=True),
                                   W.square(3, 2, U=4.0, tp=-0.3, pbc=False, n_up=2, n_dn=2)])
def test_stationary_distribution(model):
    """Symmetric proposal + Metropolis ratio: visit frequencies -> exp(-b E)/Z."""
    beta = 0.5
    k = fock.sector_keys(model.n_orb, model.n_up, model.n_dn)
    E = fock.diagonal(k, model)
    p = np.exp(-beta * (E - E.min()))
    p /= p.sum()
    steps = 4_000_000
    counts = sampler.chain_histogram(model, W.neel_start(model), 123, 10_000, steps, k, beta)
    # thin by the autocorrelation: compare with a generous effective sample size
    n_eff = steps / 50
    f = counts / steps
    chi2 = n_eff * np.sum((f - p) ** 2 / p)
    dof = len(k) - 1
    assert chi2 < stats.chi2.ppf(0.999, dof), (chi2, dof)
    # a chain that ignored the acceptance would be uniform: that must fail
    u = np.full(len(k), 1.0 / len(k))
    assert n_eff * np.sum((f - u) ** 2 / u) > stats.chi2.ppf(0.999, dof)


def test_chain_stops_at_n_f_and_respects_cap():
    m = W.config_c1()["model"]
    a, s = sampler.chain_c(m, W.neel_start(m), 4, 100, 10, 10**6)
    assert len(a) == 100
    b, s2 = sampler.chain_c(m, W.neel_start(m), 4, 4900, 10, 2000)
    assert s2 == 2000 and len(b) < 4900


# --- the paper's step sampler (Sec. Subspace of the ground state) ----------
def test_step_sampler_python_and_numpy_agree():
    for m, nf, beta in [(W.config_c1()["model"], 2000, 0.2), (W.chain(4, U=8.0, mu=4.0), 18, 0.2),
                        (W.impurity_plaquette_bath(3), 5000, 0.2)]:
        st = W.neel_start(m)
        a, sa = sampler.bfs_python(m, st, 7, beta, nf, 1000)
        b, sb = sampler.bfs_numpy(m, st, 7, beta, nf, 1000)
        assert sa == sb and np.array_equal(a, b) and len(a) == nf
        fock.check_sector(a, m)
        assert W.neel_start(m) in set(int(k) for k in a)


def test_step_sampler_limits():
    m = W.config_c1()["model"]
    st = W.neel_start(m)
    # beta = 0 accepts every hop: the whole (connected) sector is reached
    a, _ = sampler.bfs_numpy(m, st, 1, 0.0, 4900, 1000)
    assert np.array_equal(a, fock.sector_keys(8, 4, 4))
    # beta = 0: the first steps are breadth-first shells around the start state
    a2, s2 = sampler.bfs_numpy(m, st, 1, 0.0, 10**9, 2)
    one = set()
    H = ham.build_csr(fock.sector_keys(8, 4, 4), m)
    keys = fock.sector_keys(8, 4, 4)
    i0 = int(np.searchsorted(keys, np.uint64(st)))
    d1 = set(H[i0].indices) | {i0}
    d2 = set(j for i in d1 for j in H[i].indices) | d1
    assert set(np.searchsorted(keys, a2)) == d2
    # huge beta: only states without double occupation are accepted
    a3, _ = sampler.bfs_numpy(m, st, 1, 1e3, 4900, 40)
    assert np.all(fock.double_occupation(a3) == 0)


def test_step_sampler_preacceptance():
    """Pre-accepted low-n_U levels (Sec. Monte Carlo sampling): the n_U = 0
    level of a half-filled N-site cluster holds C(N, N_up) states (one
    electron per site, any spin pattern with N_up ups); a level above every
    n_U takes the whole sector without a step; the two implementations agree;
    the result keeps every pre-accepted state and adds only higher-n_U ones."""
    import math
    m = W.chain(8, U=8.0, mu=4.0)
    P = sampler.preaccepted(m, 1)
    assert len(P) == math.comb(8, 4) and np.all(fock.double_occupation(P) == 0)
    P2 = sampler.preaccepted(m, 2)
    assert len(P2) == math.comb(8, 4) + 8 * 7 * math.comb(6, 3)
    full, st = sampler.bfs_numpy(m, W.neel_start(m), 1, 0.2, 4900, 50, pre_level=9)
    assert st == 0 and np.array_equal(full, fock.sector_keys(8, 4, 4))
    for lvl, nf in ((1, 600), (2, 2500), (2, 1000)):
        a, sa = sampler.bfs_python(m, W.neel_start(m), 3, 0.2, nf, 200, pre_level=lvl)
        b, sb = sampler.bfs_numpy(m, W.neel_start(m), 3, 0.2, nf, 200, pre_level=lvl)
        assert sa == sb and np.array_equal(a, b) and len(a) == nf
        Pl = sampler.preaccepted(m, lvl)
        if nf <= len(Pl):           # first nf of the pre-accepted set, no step
            assert sa == 0 and np.array_equal(a, np.sort(Pl[:nf]))
        else:
            assert np.all(np.isin(Pl, a)) and np.all(fock.double_occupation(a[~np.isin(a, Pl)]) >= lvl)


@pytest.mark.parametrize("U", [4.0, 8.0])
def test_step_sampler_acceptance_law(U):
    """Acceptance of the step sampler (Eq. boltzmann_factor): a proposal is
    kept with probability min(1, exp(-beta U n_U)), n_U the double occupation
    of the proposed state.  First step from a state with one doubly occupied
    site, so the proposals fall in the classes n_U = 0, 1 and 2; over many
    seeds the kept fraction of each class must match exp(-beta U n_U) (a law
    without U, or one indexed by the change of n_U, fails)."""
    beta = 0.2
    m = W.chain(8, U=U, mu=U / 2, pbc=True)
    up, dn = 0b01010110, 0b10101010                  # site 1 doubly occupied, site 0 empty
    start = (up << 32) | dn
    # the proposals of the first step and their classes
    props = []
    for (i, j, _) in m.bonds:
        for spin in (0, 1):
            for src, dst in ((i, j), (j, i)):
                s = up if spin == 0 else dn
                if not (s >> src) & 1 or (s >> dst) & 1:
                    continue
                s2 = s ^ ((1 << src) | (1 << dst))
                y = (s2 << 32) | dn if spin == 0 else (up << 32) | s2
                props.append((y, bin((y >> 32) & y & 0xFF).count("1")))
    classes = sorted(set(k for _, k in props))
    assert classes == [0, 1, 2]
    tried = {k: 0 for k in classes}
    kept = {k: 0 for k in classes}
    for seed in range(2500):
        a, st = sampler.bfs_numpy(m, start, seed, beta, 10**9, 1)
        got = set(int(k) for k in a)
        for y, k in props:
            tried[k] += 1
            kept[k] += y in got
    for k in classes:
        p = np.exp(-beta * U * k)
        f = kept[k] / tried[k]
        sd = np.sqrt(max(p * (1 - p), 1e-12) / tried[k])
        assert abs(f - p) <= 4.5 * sd + 1e-12, (k, f, p)
        if k > 0:
            # the same law without U, and one counting the change of n_U
            for wrong in (np.exp(-beta * k), np.exp(-beta * U * (k - 1))):
                assert abs(f - wrong) > 8 * sd, (k, f, wrong)
