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
