"""GPU parity of mcd_lanczos_ground against the oracle (E0 to 1e-10 relative,
ground state overlap) and the paper's printed full-ED energies."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fock, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_energies.json")))


def _oracle(keys, m, tol=1e-13, reorth=True, max_iter=500):
    H = ham.build_csr(keys, m)
    return H, lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=tol, max_iter=max_iter,
                                reorth=reorth)


def _cases():
    c1 = W.config_c1()
    m1 = c1["model"]
    k1s, _ = sampler.chain_c(m1, W.neel_start(m1), c1["seed"], c1["n_f"], c1["burn_in"],
                             c1["max_steps"])
    imp = W.impurity_plaquette_bath(3)
    ki, _ = sampler.chain_c(imp, W.neel_start(imp), 9, 20000, 1000, 10**7)
    return {
        "c1_full": (m1, fock.sector_keys(8, 4, 4)),
        "c1_chain": (m1, k1s),
        "imp_chain": (imp, ki),
        "two_site": (W.chain(2, U=4.0, pbc=False, n_up=1, n_dn=1), fock.sector_keys(2, 1, 1)),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("storage,store,kern", [("csr", True, "stream"), ("otf", False, None),
                                                ("csr", True, "rowchunk"),
                                                ("csr", False, "merge"), ("csr", True, "stream_xcd")])
def test_e0_and_ground_state(name, storage, store, kern):
    torch, mcd = require_gpu()
    m, keys = CASES[name]
    log_case("lanczos", case=name, storage=storage, store=store, kernel=kern, n=len(keys))
    H, ro = _oracle(keys, m)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
    if kern:
        op.set_kernel(kern)
    e0, psi, a, b, info = mcd.lanczos_ground(op, max_iter=400, tol=1e-12, seed=11,
                                              store_vectors=store)
    assert abs(e0 - ro["e0"]) <= 1e-10 * abs(ro["e0"])
    p = psi.cpu().numpy()
    assert abs(np.linalg.norm(p) - 1) < 1e-12
    assert abs(abs(p @ ro["psi0"]) - 1.0) < 1e-8
    assert np.linalg.norm(H @ p - e0 * p) < 1e-5
    # the first Lanczos coefficient pins the start vector (splitmix64 of key ^ seed)
    v0 = lz.start_vector(keys, 11)
    assert abs(a[0] - (v0 @ (H @ v0)) / (v0 @ v0)) <= 1e-13 * max(1, abs(a[0]))
    if name == "two_site":
        assert abs(e0 - (2.0 - math.sqrt(4.0 + 4.0))) < 1e-12
    op.close()


@pytest.mark.parametrize("name", ["c1_full", "c1_chain", "imp_chain"])
@pytest.mark.parametrize("storage,store", [("csr", True), ("otf", False)])
def test_float32_krylov_vectors_refined_e0(name, storage, store):
    """Float32 Krylov vectors with float64 coefficients, then one float64
    product for the Rayleigh quotient of the Ritz vector: E0 within 1e-9 of
    the oracle (the quotient's error is second order in the float32-level
    error of the vector), psi0 overlap to 1e-6, and the reported residual is
    the true float64 residual ||H psi - E0 psi||."""
    torch, mcd = require_gpu()
    m, keys = CASES[name]
    log_case("lanczos_f32", case=name, storage=storage, store=store, n=len(keys))
    H, ro = _oracle(keys, m)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
    e0, psi, a, b, info = mcd.lanczos_ground(op, max_iter=400, tol=1e-9, seed=11,
                                              store_vectors=store, precision="f32")
    p = psi.cpu().numpy()
    print("[f32] E0 err", abs(e0 - ro["e0"]) / abs(ro["e0"]), "resid", info.residual, flush=True)
    assert abs(e0 - ro["e0"]) <= 1e-9 * abs(ro["e0"])
    assert abs(np.linalg.norm(p) - 1) < 1e-12
    assert abs(abs(p @ ro["psi0"]) - 1.0) < 1e-6
    assert abs(e0 - p @ (H @ p)) <= 1e-12 * abs(e0)
    assert abs(info.residual - np.linalg.norm(H @ p - e0 * p)) <= 1e-6 * max(info.residual, 1e-9)
    # the start vector is the float64 one rounded to float32
    v0 = lz.start_vector(keys, 11).astype(np.float32).astype(np.float64)
    assert abs(a[0] - (v0 @ (H @ v0)) / (v0 @ v0)) <= 1e-6 * max(1, abs(a[0]))
    op.close()


def test_paper_energies_on_gpu():
    """Full-ED energies printed in the paper's appendix tables (truncated to 4 decimals)."""
    torch, mcd = require_gpu()
    cases = [(W.chain(8, U=8.0, mu=4.0), GOLD["table_1D_energies_f1"]["8"]),
             (W.chain(12, U=8.0, mu=4.0), GOLD["table_1D_energies_f1"]["12"]),
             (W.square(4, 2, U=8.0, mu=4.0, pbc=True), GOLD["table_2D_energies_f1"]["2x4"]),
             (W.superlattice((4, 0), (1, 3), U=8.0, mu=4.0), GOLD["table_2D_energies_f1"]["12"])]
    for m, want in cases:
        log_case("paper_energy", model=m.name)
        k, _ = mcd.basis_build(m, "full")
        op = mcd.Operator(m, k)
        e0, _, _, _, info = mcd.lanczos_ground(op, max_iter=400, tol=1e-11, want_psi=False)
        assert math.trunc(e0 / m.n_orb * 1e4) / 1e4 == want
        op.close()


def test_variational_order_nested_chain_bases():
    """Truncation raises the energy: a chain basis that is a prefix of a longer
    run (same seed) gives E0 >= the longer run's E0."""
    torch, mcd = require_gpu()
    m = W.config_c1()["model"]
    st = W.neel_start(m)
    last = -np.inf
    for nf in (4000, 2000, 800, 200):
        k, _ = mcd.basis_build(m, "chain", start_key=st, seed=1, beta_s=0.5, burn_in=1000,
                               max_steps=10**7, n_f=nf)
        op = mcd.Operator(m, k)
        e0, *_ = mcd.lanczos_ground(op, max_iter=400, tol=1e-12, want_psi=False)
        assert e0 >= last - 1e-10
        last = e0
        op.close()


def test_c2_full_size_e0():
    """C2 at full size (4x4 t-t', 4M chain states).  (a) 200 steps from the same
    start vector: GPU and oracle Ritz values agree to 1e-10 relative (same
    Krylov space, float64, no reorthogonalisation on either side).  (b) run to
    a 1e-10 residual: E0 agrees with the oracle's converged E0 to 1e-10."""
    torch, mcd = require_gpu()
    c = W.config_c2()
    m = c["model"]
    keys, _ = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                              c["max_steps"])
    log_case("lanczos_c2", n=len(keys))
    H = ham.build_csr(keys, m)
    v0 = lz.start_vector(keys, 11)
    r200 = lz.lanczos_ground(H, v0, tol=0.0, max_iter=200, reorth=False)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys))
    e200, *_ = mcd.lanczos_ground(op, max_iter=200, tol=0.0, seed=11, min_iter=200,
                                  want_psi=False)
    print("[c2] E0(200) gpu", e200, "oracle", r200["e0"], flush=True)
    assert abs(e200 - r200["e0"]) <= 1e-10 * abs(r200["e0"])
    rc = lz.lanczos_ground(H, v0, tol=1e-10, max_iter=1500, reorth=False)
    ec, psi, _, _, info = mcd.lanczos_ground(op, max_iter=1500, tol=1e-10, seed=11)
    print("[c2] E0(conv) gpu", ec, info.iters, "oracle", rc["e0"], rc["iters"], flush=True)
    assert abs(ec - rc["e0"]) <= 1e-10 * abs(rc["e0"])
    # (c) float32 Krylov vectors + float64 Rayleigh-quotient refinement: 1e-8
    e32, p32, _, _, i32 = mcd.lanczos_ground(op, max_iter=1500, tol=1e-9, seed=11,
                                             precision="f32")
    err = abs(e32 - rc["e0"]) / abs(rc["e0"])
    print("[c2] E0 f32+refine", e32, i32.iters, "rel err", err, "resid", i32.residual, flush=True)
    assert err <= 1e-8
    op.close()


def test_c5_full_size_200_step_ritz_value():
    """C5 at full size (4x8 t-t', 50M chain states): the GPU's Ritz value
    after 200 steps from the seed-11 start vector against the oracle's
    (tests/golden/c5_ritz200.json, written by tests/golden/make_c5_ritz.py
    from the oracle alone: same Krylov space, float64, no
    reorthogonalisation on either side), to 1e-10 relative; the first
    coefficient a_0 to 1e-12."""
    torch, mcd = require_gpu()
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_ritz200.json")))
    c = W.config_c5()
    m = c["model"]
    log_case("lanczos_c5", n_f=c["n_f"])
    kd, steps = mcd.basis_build(m, "chain", start_key=W.neel_start(m), seed=c["seed"],
                                beta_s=c["beta_s"], burn_in=c["burn_in"],
                                max_steps=c["max_steps"], n_f=c["n_f"])
    assert kd.numel() == gold["n"] and steps == gold["chain_steps"]
    op = mcd.Operator(m, kd, storage="csr")
    e200, _, a, _, info = mcd.lanczos_ground(op, max_iter=200, tol=0.0, seed=11, min_iter=200,
                                             want_psi=False, store_vectors=False)
    print("[c5] E0(200) gpu", e200, "oracle", gold["e0_200"], flush=True)
    assert info.iters == 200
    assert abs(a[0] - gold["alpha_0"]) <= 1e-12 * abs(gold["alpha_0"])
    assert abs(e200 - gold["e0_200"]) <= 1e-10 * abs(gold["e0_200"])
    op.close()
