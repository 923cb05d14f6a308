"""The allocation-free contraction (mcd_hamiltonian_contract_noalloc, fixed
device scratch) against mcd_hamiltonian_contract (workspace) through the C
ABI: bit-identical derivatives on two calls in a row, the second on a
smaller basis (the fixed scratch keeps the first call's partials, which the
second must overwrite before reading)."""
import numpy as np
import pytest

import workloads as W
from oracle import fock, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu


def test_noalloc_contract_matches_workspace_contract():
    torch, mcd = require_gpu()
    m1 = W.impurity_plaquette_bath(3)
    k1, _ = sampler.chain_c(m1, W.neel_start(m1), 9, 20000, 500, 10**7)
    m2 = W.config_c1()["model"]
    k2 = fock.sector_keys(8, 4, 4)[::3]            # a smaller basis (1634 states)
    for m, keys in ((m1, k1), (m2, k2)):
        log_case("noalloc_contract", n=len(keys))
        op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
        rng = np.random.default_rng(len(keys))
        a = torch.from_numpy(rng.uniform(-1, 1, len(keys))).cuda()
        b = torch.from_numpy(rng.uniform(-1, 1, len(keys))).cuda()
        ref = op.contract(a, b)
        got = op.contract_noalloc(a, b)
        for r, g in zip(ref, got):
            assert np.array_equal(r, g)
        # Hellmann-Feynman form (a = b) as well
        ref2 = op.contract(a)
        got2 = op.contract_noalloc(a)
        for r, g in zip(ref2, got2):
            assert np.array_equal(r, g)
        op.close()
