"""No read of unwritten device memory on the solver paths.

With the workspace flag MCD_WS_POISON every floating-point piece the library
takes (vectors, Krylov blocks, Gram partials, coefficient and recurrence
stores, reduction scratch, the operator's diagonal) is filled with NaN bytes
when it is taken.  A kernel that read such a piece before writing it would
turn the result into NaN or change it; correct code gives results bit for bit
those of the same calls without the flag.  The same operator serves both
sides (an operator built under the flag had its own pieces poisoned), so the
product kernel and its row order are the same; every result is also checked
to be finite and close to the oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import green as gr, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu
OM = W.matsubara(16, 50.0)


@pytest.fixture
def poisoned():
    torch, mcd = require_gpu()
    mcd.release_scratch()
    old = mcd.workspace_debug(mcd.WS_POISON)
    try:
        yield torch, mcd
    finally:
        mcd.workspace_debug(old)
        mcd.release_scratch()


def _both(mcd, call):
    """call() under the poison flag, then again without it."""
    mcd.release_scratch()
    mcd.workspace_debug(mcd.WS_POISON)
    a = call()
    mcd.release_scratch()
    mcd.workspace_debug(0)
    b = call()
    mcd.workspace_debug(mcd.WS_POISON)
    return a, b


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _c1_chain():
    c = W.config_c1()
    m = c["model"]
    k, _ = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"], c["max_steps"])
    return m, k


def _impurity(seed=6, n_f=4000):
    m = W.impurity_plaquette_bath(seed)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 2, n_f, 500, 10**7)
    return m, keys


@pytest.mark.parametrize("storage", ["csr", "otf"])
def test_poison_operator_and_lanczos(poisoned, storage):
    torch, mcd = poisoned
    m, keys = _c1_chain()
    log_case("poison_lanczos", n=len(keys), storage=storage)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)   # built poisoned
    try:
        H = ham.build_csr(keys, m)
        ro = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13, max_iter=600)
        d = op.diagonal().cpu().numpy()
        assert np.isfinite(d).all() and np.array_equal(d, H.diagonal())
        x = torch.from_numpy(np.random.default_rng(3).normal(size=len(keys))).cuda()
        y = op.apply(x).cpu().numpy()
        assert np.isfinite(y).all() and _rel(y, H @ x.cpu().numpy()) < 1e-13
        for prec, store in (("f64", True), ("f64", False), ("f32", True), ("f32", False)):
            (ea, pa, aa, ba, ia), (eb, pb, ab, bb, ib) = _both(
                mcd, lambda: mcd.lanczos_ground(op, max_iter=400, tol=1e-10, seed=11,
                                                store_vectors=store, precision=prec))
            assert np.isfinite(ea) and ea == eb and ia.iters == ib.iters, (prec, store)
            assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy()), (prec, store)
            assert np.array_equal(aa, ab) and np.array_equal(ba, bb)
            assert abs(ea - ro["e0"]) <= 1e-9 * abs(ro["e0"]), (prec, store)
        a = torch.from_numpy(ro["psi0"]).cuda()
        ca, cb = _both(mcd, lambda: op.contract(a))
        for u, v in zip(ca, cb):
            u, v = np.asarray(u), np.asarray(v)
            assert np.isfinite(u).all() and np.array_equal(u, v)
    finally:
        op.close()


@pytest.mark.parametrize("case", ["f64_r2_p8", "f64_r0_p4", "f32_r0_p8", "f32_r1_p16",
                                  "f64_percol_p4", "f32_wt"])
def test_poison_band_green(poisoned, case):
    torch, mcd = poisoned
    m, keys = _c1_chain()
    H = ham.build_csr(keys, m)
    r = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13)
    e0, psi = r["e0"], r["psi0"]
    sel = {"p8": ([0, 1, 2, 3] * 2, [0] * 4 + [1] * 4), "p4": ([0, 1, 2, 3], [0] * 4),
           "p16": (list(range(8)) * 2, [0] * 8 + [1] * 8)}
    prec, rest = case.split("_", 1)
    kw = dict(max_blocks=30, precision=prec, g_tol=1e-9 if prec == "f64" else 1e-6)
    if rest == "wt":
        orbs, spins = sel["p8"]
        kw.update(w_t=0.99, reorth=0)
    else:
        mode, width = rest.split("_")
        orbs, spins = sel[width]
        if mode == "percol":
            kw.update(per_column=True, reorth=2)
        else:
            kw.update(reorth=int(mode[1]))
    log_case("poison_green", case=case, n=len(keys))
    kd = mcd.keys_from_numpy(keys)
    pt = torch.from_numpy(psi).cuda()
    (Ga, ia), (Gb, ib) = _both(
        mcd, lambda: mcd.band_lanczos_green(m, kd, pt, e0, orbs, spins, OM, **kw))
    assert np.isfinite(Ga).all() and ia.iters == ib.iters
    if kw.get("per_column"):
        # the per-column form tunes the product kernel of each sector's operator
        assert _rel(Ga, Gb) <= 1e-12
    else:
        assert np.array_equal(Ga, Gb)
    if kw.get("w_t", 1.0) == 1.0 and prec == "f64":
        Go = np.zeros_like(Ga)
        for s in (0, 1):
            q = [i for i in range(len(orbs)) if spins[i] == s]
            if q:
                Gs = gr.green_mcd(keys, m, psi, e0, [orbs[i] for i in q], s, OM,
                                  max_dim=len(q) * ia.iters)
                Go[np.ix_(range(len(OM)), q, q)] = Gs
        assert _rel(Ga, Go) <= 1e-6


@pytest.mark.parametrize("prec,keep", [("f64", False), ("f32", False), ("f32", True)])
def test_poison_green_vjp(poisoned, prec, keep):
    torch, mcd = poisoned
    m, keys = _impurity()
    kd = mcd.keys_from_numpy(keys)
    op = mcd.Operator(m, kd, storage="csr")
    e0, psi, *_ = mcd.lanczos_ground(op, max_iter=600, tol=1e-12, seed=11)
    op.close()
    orbs, spins = [0, 1, 2, 3], [0, 0, 1, 1]
    rng = np.random.default_rng(4)
    Gb = rng.normal(size=(len(OM), 4, 4)) + 1j * rng.normal(size=(len(OM), 4, 4))
    kw = dict(max_blocks=60, reorth=1, g_tol=1e-8, precision=prec)
    log_case("poison_vjp", n=len(keys), prec=prec, keep=keep)

    def call():
        if not keep:
            return mcd.band_green_vjp(m, kd, psi, e0, orbs, spins, OM, Gb, e0_bar=0.3, **kw)
        G, info, kept = mcd.band_lanczos_green(m, kd, psi, e0, orbs, spins, OM, keep=True, **kw)
        try:
            return (G,) + tuple(mcd.band_green_vjp(m, kd, psi, e0, orbs, spins, OM, Gb,
                                                   e0_bar=0.3, keep=kept, **kw)[:3])
        finally:
            kept.close()
    a, b = _both(mcd, call)
    for u, v in zip(a[:4] if keep else a[:3], b[:4] if keep else b[:3]):
        assert np.isfinite(u).all() and np.array_equal(u, v)


def test_poison_batched_ground_states_and_green(poisoned):
    torch, mcd = poisoned
    inst = [_impurity(3 + k, n_f) for k, n_f in enumerate((3000, 800, 5000))]
    log_case("poison_batch", sizes=[len(k) for _, k in inst])
    kds = [mcd.keys_from_numpy(k) for _, k in inst]
    ops = [mcd.Operator(m, kd, storage="csr") for (m, _), kd in zip(inst, kds)]
    try:
        (ea, pa, ia, _), (eb, pb, ib, _) = _both(
            mcd, lambda: mcd.batch_lanczos_ground(ops, max_iter=400, tol=1e-12, seed=11))
        assert ea == eb and ia == ib and all(np.isfinite(ea))
        for u, v in zip(pa, pb):
            assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())
        orbs, spins = [0, 1, 2, 3] * 2, [0] * 4 + [1] * 4
        (Ga, _), (Gb, _) = _both(
            mcd, lambda: mcd.batch_band_green([m for m, _ in inst], kds, pa, ea, orbs, spins, OM,
                                              max_blocks=40, precision="f32", reorth=0,
                                              g_tol=1e-6))
        for u, v in zip(Ga, Gb):
            assert np.isfinite(u).all() and np.array_equal(u, v)
    finally:
        for op in ops:
            op.close()


def test_poison_flag_fills_unwritten_pieces(poisoned):
    """Control: the flag does fill pieces.  A Lanczos solve that stores up to
    400 vectors but converges in far fewer leaves the rest of its store as
    taken: all-ones 8-byte words with the flag, none without it (the buffer is
    zeroed first, and a solve writes no all-ones word: that is a NaN)."""
    torch, mcd = poisoned
    m, keys = _c1_chain()
    n = len(keys)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
    try:
        counts = []
        for flag in (mcd.WS_POISON, 0):
            mcd.release_scratch()
            mcd.workspace_debug(flag)
            ws = mcd.scratch(64 << 20)
            ws.buf.zero_()
            _, _, _, _, info = mcd.lanczos_ground(op, max_iter=400, tol=1e-10, seed=11,
                                                  store_vectors=True)
            torch.cuda.synchronize()
            assert mcd.scratch() is ws and info.iters < 300
            counts.append(int((ws.buf.view(torch.int64) == -1).sum().item()))
        assert counts[0] >= (400 - info.iters - 1) * n and counts[1] == 0, counts
    finally:
        mcd.workspace_debug(mcd.WS_POISON)
        op.close()
