"""GPU derivatives: mcd_hamiltonian_contract (<a| dH~/dtheta |b>) and the
differentiable ground-state energy, against the oracle's derivative operators
and central finite differences of the oracle's E0."""
import numpy as np
import pytest

import workloads as W
from oracle import derivatives as dv, fock, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu


def _imp(seed=4, nf=6000):
    m = W.impurity_plaquette_bath(seed)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 3, nf, 500, 10**7)
    return m, keys


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("storage", ["csr", "otf"])
def test_contract_bilinear_vs_oracle(storage):
    torch, mcd = require_gpu()
    m, keys = _imp()
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=len(keys)), rng.normal(size=len(keys))
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
    got = op.contract(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    ref = dv.contract(keys, m, a, b)
    for g, r in zip(got, ref):
        assert _rel(g, r) <= 1e-12
    op.close()


def test_hellmann_feynman_all_33_parameters():
    """dE0/dtheta for theta = (eps_b, V_ib, U) through torch autograd, against
    the oracle's Hellmann-Feynman values (all 33) and its central finite
    differences (h = 1e-5) on six of them."""
    torch, mcd = require_gpu()
    from paper_2509_22975_amd.autograd import ground_energy, impurity_parameters
    m, keys = _imp()
    theta0, expand = impurity_parameters(m)
    assert len(theta0) == 33
    kd = mcd.keys_from_numpy(keys)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    t, U, eps = expand(theta)
    e0 = ground_energy(m, kd, t, U, eps)
    e0.backward()
    g = theta.grad.numpy()

    def oracle_e0(th):
        tt, uu, ee = [x.detach().numpy() for x in expand(torch.tensor(th, dtype=torch.float64))]
        mm = m.with_params(bonds=[(b[0], b[1], float(v)) for b, v in zip(m.bonds, tt)], U=uu, eps=ee)
        H = ham.build_csr(keys, mm)
        return lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13, max_iter=800)

    r = oracle_e0(theta0)
    assert abs(e0.item() - r["e0"]) <= 1e-10 * abs(r["e0"])
    dt, dU, de = dv.contract(keys, m, r["psi0"], r["psi0"])
    hyb = [q for q, b in enumerate(m.bonds) if b[1] >= 4]
    imp = [0, 1, 2, 3]
    hf = np.concatenate([de[4:], dt[hyb], [dU[imp].sum() - 0.5 * de[imp].sum()]])
    assert np.max(np.abs(g - hf)) <= 1e-8 * max(1.0, np.max(np.abs(hf)))
    idx = [0, 5, 8, 20, 31, 32]
    fd = dv.central_difference(lambda th: oracle_e0(th)["e0"], theta0, idx)
    print("[grad] fd", fd, "gpu", g[idx], flush=True)
    assert np.max(np.abs(fd - g[idx])) < 1e-6
