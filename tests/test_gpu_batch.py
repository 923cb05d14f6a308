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
