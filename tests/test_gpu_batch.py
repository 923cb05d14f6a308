"""Batched ground states (mcd_batch_lanczos_ground): several bath instances of
uneven basis size in one lockstep solve, against single solves and the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import fock, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu


def _instances():
    out = []
    for k, nf in enumerate((6000, 20000, 1500, 12000, 40)):
        m = W.impurity_plaquette_bath(3 + k)
        keys, _ = sampler.chain_c(m, W.neel_start(m), 9 + k, nf, 500, 10**7)
        out.append((m, keys))
    out.append((W.config_c1()["model"], fock.sector_keys(8, 4, 4)))
    return out


def test_batch_matches_single_and_oracle():
    torch, mcd = require_gpu()
    inst = _instances()
    log_case("batch", sizes=[len(k) for _, k in inst])
    ops = [mcd.Operator(m, mcd.keys_from_numpy(k), storage="csr") for m, k in inst]
    e0s, psis, its, info = mcd.batch_lanczos_ground(ops, max_iter=400, tol=1e-12, seed=11,
                                                    check_every=10)
    assert info.converged
    for i, ((m, keys), op) in enumerate(zip(inst, ops)):
        e1, p1, _, _, si = mcd.lanczos_ground(op, max_iter=400, tol=1e-12, seed=11,
                                              check_every=10)
        H = ham.build_csr(keys, m)
        ro = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13, max_iter=600)
        assert abs(e0s[i] - ro["e0"]) <= 1e-10 * abs(ro["e0"]), i
        assert abs(e0s[i] - e1) <= 1e-12 * abs(e1), i
        p = psis[i].cpu().numpy()
        assert abs(abs(p @ ro["psi0"]) - 1.0) < 1e-8, i
        assert its[i] == si.iters, (i, its[i], si.iters)
    for op in ops:
        op.close()


def test_batch_single_instance_and_step_cap():
    torch, mcd = require_gpu()
    m, keys = _instances()[1]
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
    e0s, _, its, info = mcd.batch_lanczos_ground([op], max_iter=37, tol=0.0, seed=5,
                                                 check_every=10, want_psi=False)
    e1, _, _, _, si = mcd.lanczos_ground(op, max_iter=37, tol=0.0, seed=5, check_every=10,
                                          want_psi=False)
    assert not info.converged and its[0] == 37 and si.iters == 37
    assert abs(e0s[0] - e1) <= 1e-12 * abs(e1)
    op.close()


def test_batch_green_equals_single_and_oracle():
    """mcd_batch_band_green on several instances (all runs in lockstep) returns exactly
    what mcd_band_lanczos_green returns per instance; one instance is also
    checked against the oracle (same Krylov space, float64)."""
    torch, mcd = require_gpu()
    from oracle import green as gr
    inst = _instances()[:5]
    om = W.matsubara(16, 50.0)
    orbs, spins = [0, 1, 2, 3, 0, 1, 2, 3], [0, 0, 0, 0, 1, 1, 1, 1]
    log_case("batch_green", sizes=[len(k) for _, k in inst])
    kds, psis, e0s = [], [], []
    for m, keys in inst:
        kd = mcd.keys_from_numpy(keys)
        op = mcd.Operator(m, kd, storage="csr")
        e0, psi, _, _, _ = mcd.lanczos_ground(op, max_iter=600, tol=1e-12, seed=11)
        op.close()
        kds.append(kd)
        psis.append(psi)
        e0s.append(e0)
    for prec, reorth in (("f64", 2), ("f32", 0)):
        Gb, info = mcd.batch_band_green([m for m, _ in inst], kds, psis, e0s, orbs, spins, om,
                                        max_blocks=12, precision=prec,
                                        reorth=reorth)
        assert info.krylov_dim > 0
        for i, (m, keys) in enumerate(inst):
            G1, _ = mcd.band_lanczos_green(m, kds[i], psis[i], e0s[i], orbs, spins, om,
                                           max_blocks=12, precision=prec, reorth=reorth)
            assert np.array_equal(Gb[i], G1), (prec, i)
    # instance 1 against the oracle (up spin block), float64
    m, keys = inst[1]
    G1, _ = mcd.band_lanczos_green(m, kds[1], psis[1], e0s[1], orbs, spins, om, max_blocks=12,
                                   reorth=2)
    psi = psis[1].cpu().numpy()
    ref = gr.green_mcd(keys, m, psi, e0s[1], [0, 1, 2, 3], 0, om, max_dim=4 * 12)
    assert np.max(np.abs(G1[:, :4, :4] - ref)) <= 1e-9 * np.max(np.abs(ref))
    # an invalid selection for one instance is rejected before any work
    bad = [m for m, _ in inst]
    with pytest.raises(mcd.McdError):
        mcd.batch_band_green(bad, kds, psis, e0s, [0, 40], [0, 0], om)
