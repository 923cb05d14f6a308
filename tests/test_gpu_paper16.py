"""The paper's full-ED energies at 16 sites, computed on the GPU (f = 1, the
whole 165,636,900-state sector; too large for the CPU oracle, so the pins
are the printed values, truncated to 4 decimals as the tables are)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_energies.json")))


def trunc4(x):
    return math.trunc(x * 1e4) / 1e4


def _e0(mcd, m):
    k, _ = mcd.basis_build(m, "full")
    assert k.numel() == GOLD["table_reduce_green_f1_wt1"]["F_size"]
    op = mcd.Operator(m, k, storage="csr", validate=False)
    info = op.info()
    e0, _, _, _, si = mcd.lanczos_ground(op, max_iter=600, tol=1e-9, want_psi=False,
                                         check_every=20)
    print(f"[paper16] {m.name} n={info['n']} nnz={info['nnz']} E0={e0:.10f} "
          f"E0/N={e0 / m.n_orb:.8f} iters={si.iters} solve={si.solve_ms:.0f} ms", flush=True)
    op.close()
    del k
    return e0


def test_16_site_ring_and_mu_shift():
    torch, mcd = require_gpu()
    m = W.chain(16, t=1.0, U=8.0, mu=4.0, pbc=True)
    log_case("paper16_ring")
    e0 = _e0(mcd, m)
    assert trunc4(e0 / 16) == GOLD["table_1D_energies_f1"]["16"]
    # mu = 2.0 keeps the half-filled ground state: E/N shifts by (4 - 2) N_e / N_c
    assert trunc4((e0 + 2.0 * 16) / 16) == GOLD["table_mu_energies_ED_16site"]["2.0"]
    assert trunc4((e0 + 2.4 * 16) / 16) == GOLD["table_mu_energies_ED_16site"]["1.6"]


def test_16_site_square():
    torch, mcd = require_gpu()
    m = W.square(4, 4, t=1.0, U=8.0, mu=4.0, pbc=True)
    log_case("paper16_square")
    e0 = _e0(mcd, m)
    assert trunc4(e0 / 16) == GOLD["table_2D_energies_f1"]["4x4"]


def test_16_site_ring_f005_sampled_pipeline():
    """The paper's f = 0.05 pipeline on the 16-site ring: step sampler
    (beta = 0.2, N_f = 8,281,845), ground state, w_t = 0.999 cut, F~+.  The
    paper's random stream is not ours, so the printed values are matched
    within the spread a different seed gives: E/N_c within 2e-3 of -4.3187,
    |F~| after the cut and |F~+| within 10% of ~806,000 and ~4,200,000."""
    torch, mcd = require_gpu()
    m = W.chain(16, t=1.0, U=8.0, mu=4.0, pbc=True)
    log_case("paper16_f005")
    keys, _ = mcd.basis_build(m, "steps", start_key=W.neel_start(m), seed=1, beta_s=0.2,
                              max_steps=100000, n_f=GOLD["N_f_16site_f005"])
    assert keys.numel() == GOLD["N_f_16site_f005"]
    op = mcd.Operator(m, keys, storage="csr")
    e0, psi, _, _, _ = mcd.lanczos_ground(op, max_iter=2000, tol=1e-9, seed=11)
    op.close()
    assert abs(e0 / 16 - GOLD["table_1D_energies_f005"]["16"]) < 2e-3
    # variational: above the full-sector energy
    assert e0 / 16 > GOLD["table_1D_energies_f1"]["16"] - 1e-4
    # F~+ for all 16 sites (the table's subspace): one selection of every site
    sizes = GOLD["table_reduce_green_f005_wt0999"]
    G, gi = mcd.band_lanczos_green(m, keys, psi, e0, list(range(16)), [0] * 16,
                                   np.array([0.0]), max_blocks=1, precision="f32", reorth=0,
                                   w_t=0.999, eta=0.05)
    assert abs(gi.n_truncated / sizes["F_size_approx"] - 1) < 0.1
    assert abs(gi.n_plus / sizes["Fpm_size_approx"] - 1) < 0.1
