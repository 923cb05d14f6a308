"""The caller-owned workspace contract of the C ABI: every device buffer of
an operator, a Lanczos solve and a band Green-function call comes from a
workspace the caller hands over (a torch tensor); the size queries are exact
(the call succeeds with that many bytes and fails with MCD_E_WORKSPACE with
one 256-byte unit less, reporting a size that would serve it); results equal
those of the binding's scratch path bit for bit and the oracle to its
tolerance."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import fock, green as gr, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu
c_vp = ctypes.c_void_p


def _c1_chain():
    c = W.config_c1()
    m = c["model"]
    k, _ = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"], c["max_steps"])
    return m, k


def _op_raw(mcd, m, kd, storage, ws):
    mb = mcd._ModelBuf(m)
    h = c_vp()
    rc = mcd.lib().mcd_op_create(ctypes.byref(mb.s), c_vp(kd.data_ptr()), int(kd.numel()),
                                 mcd.STORAGE[storage], 1, ws.handle, mcd._stream(),
                                 ctypes.byref(h))
    return rc, h, mb


@pytest.mark.parametrize("storage", ["csr", "on_the_fly"])
def test_operator_workspace_query_is_exact(storage):
    torch, mcd = require_gpu()
    m, keys = _c1_chain()
    kd = mcd.keys_from_numpy(keys)
    b = mcd.operator_workspace_size(m, kd, storage, grouped=False)
    log_case("op_ws", storage=storage, bytes=b)
    ws = mcd.Workspace(b)
    rc, h, mb = _op_raw(mcd, m, kd, storage, ws)
    assert rc == 0
    st = ws.stats()
    assert st["high_water"] <= b and st["in_use"] > 0
    mcd.lib().mcd_op_destroy(h)
    assert ws.stats()["in_use"] == 0          # every piece went back
    ws.close()
    small = mcd.Workspace(b - 256)
    rc, h, mb = _op_raw(mcd, m, kd, storage, small)
    if storage == "csr":
        assert rc == mcd.MCD_E_WORKSPACE
        assert small.stats()["need"] > b - 256
    else:
        assert rc == mcd.MCD_E_WORKSPACE
    assert small.stats()["in_use"] == 0       # a failed call releases what it took
    small.close()


def test_grouped_layout_needs_its_room():
    torch, mcd = require_gpu()
    m = W.config_c1()["model"]
    keys = fock.sector_keys(8, 4, 4)
    kd = mcd.keys_from_numpy(keys)
    b = mcd.operator_workspace_size(m, kd, "csr", grouped=False)
    bg = mcd.operator_workspace_size(m, kd, "csr", grouped=True)
    assert bg > b
    info = mcd.McdOpInfo()
    for nbytes, want in ((b, 0), (bg, 1)):
        ws = mcd.Workspace(nbytes)
        rc, h, mb = _op_raw(mcd, m, kd, "csr", ws)
        assert rc == 0
        mcd.lib().mcd_op_info(h, ctypes.byref(info))
        assert (info.grouped_blocks > 0) == bool(want)
        mcd.lib().mcd_op_destroy(h)
        ws.close()


def test_apply_lanczos_green_through_caller_workspaces():
    """apply -> Lanczos -> band G, each through a workspace of exactly the
    queried size: equal to the scratch path bit for bit, and to the oracle."""
    torch, mcd = require_gpu()
    m, keys = _c1_chain()
    kd = mcd.keys_from_numpy(keys)
    op = mcd.Operator(m, kd, storage="csr")
    assert op.ws_bytes == op._ws.nbytes
    x = torch.from_numpy(W.random_vector(len(keys), 3)).cuda()
    H = ham.build_csr(keys, m)
    y = op.apply(x).cpu().numpy()
    assert np.max(np.abs(y - H @ x.cpu().numpy())) <= 1e-12 * np.max(np.abs(y))
    # Lanczos: exact workspace; one unit less fails
    cfg = mcd._lanczos_cfg(400, 10, 1e-12, 11, True, 1, "f64")
    need = ctypes.c_size_t()
    assert mcd.lib().mcd_lanczos_workspace_size(op.handle, ctypes.byref(cfg),
                                                ctypes.byref(need)) == 0
    L = mcd.lib()
    for nbytes, ok in ((need.value, True), (need.value - 256, False)):
        ws = mcd.Workspace(nbytes)
        e0 = ctypes.c_double()
        psi = torch.empty(len(keys), dtype=torch.float64, device="cuda")
        info = mcd.McdSolveInfo()
        rc = L.mcd_lanczos_ground(op.handle, ctypes.byref(cfg), None, ctypes.byref(e0),
                                  c_vp(psi.data_ptr()), None, None, ctypes.byref(info),
                                  ws.handle, mcd._stream())
        assert (rc >= 0) == ok, rc
        if not ok:
            assert rc == mcd.MCD_E_WORKSPACE and ws.stats()["in_use"] == 0
        else:
            e_ref, psi_ref, *_ = mcd.lanczos_ground(op, max_iter=400, tol=1e-12, seed=11,
                                                    store_vectors=True)
            assert e0.value == e_ref and torch.equal(psi, psi_ref)
            ro = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13)
            assert abs(e0.value - ro["e0"]) <= 1e-10 * abs(ro["e0"])
        ws.close()
    # band G: exact workspace from the query; one unit less fails
    orbs, spins = [0, 1, 2, 3] * 2, [0] * 4 + [1] * 4
    om = W.matsubara(16, 50.0)
    kw = dict(max_blocks=20, reorth=2)
    nb = mcd.band_workspace_size(m, kd, psi_ref, e_ref, orbs, spins, om, **kw)
    log_case("band_ws", bytes=nb)
    G_ref, _ = mcd.band_lanczos_green(m, kd, psi_ref, e_ref, orbs, spins, om, **kw)
    ws = mcd.Workspace(nb)
    G, info = mcd.band_lanczos_green(m, kd, psi_ref, e_ref, orbs, spins, om, ws=ws, **kw)
    assert np.array_equal(G, G_ref)
    assert ws.stats()["high_water"] <= nb and ws.stats()["in_use"] == 0
    ws.close()
    small = mcd.Workspace(nb - 256)
    with pytest.raises(mcd.McdError) as e:
        mcd.band_lanczos_green(m, kd, psi_ref, e_ref, orbs, spins, om, ws=small, **kw)
    assert e.value.code == mcd.MCD_E_WORKSPACE
    assert small.stats()["need"] >= nb - 256 and small.stats()["in_use"] == 0
    small.close()
    # the oracle (per spin sector, same Krylov space)
    psi = psi_ref.cpu().numpy()
    for s in (0, 1):
        ref = gr.green_mcd(keys, m, psi, e_ref, [0, 1, 2, 3], s, om, max_dim=4 * 20)
        sub = G[:, 4 * s:4 * s + 4, 4 * s:4 * s + 4]
        assert np.max(np.abs(sub - ref)) <= 1e-9 * np.max(np.abs(ref))
    # a kept run in a workspace of the queried size
    nk = mcd.band_workspace_size(m, kd, psi_ref, e_ref, orbs, spins, om, keep=True, **kw)
    Gk, _, kept = mcd.band_lanczos_green(m, kd, psi_ref, e_ref, orbs, spins, om, keep=True, **kw)
    assert kept._ws.nbytes == (nk + 255) // 256 * 256
    assert np.array_equal(Gk, G_ref)
    kept.close()
    op.close()


def test_batched_green_in_groups_that_fit():
    """A workspace that holds two instances at a time: the batch runs in
    groups and each G equals the single call's bit for bit."""
    torch, mcd = require_gpu()
    om = W.matsubara(8, 50.0)
    orbs, spins = [0, 1, 2, 3], [0, 0, 0, 0]
    inst = []
    for k in range(5):
        m = W.impurity_plaquette_bath(20 + k)
        keys, _ = sampler.chain_c(m, W.neel_start(m), 30 + k, 3000 + 500 * k, 500, 10**7)
        kd = mcd.keys_from_numpy(keys)
        op = mcd.Operator(m, kd, storage="csr")
        e0, psi, *_ = mcd.lanczos_ground(op, max_iter=600, tol=1e-12, seed=11)
        op.close()
        inst.append((m, kd, psi, e0))
    kw = dict(max_blocks=16, precision="f32", reorth=1)
    singles = [mcd.band_lanczos_green(m, kd, psi, e0, orbs, spins, om, **kw)[0]
               for m, kd, psi, e0 in inst]
    sizes = [mcd.band_workspace_size(m, kd, psi, e0, orbs, spins, om, **kw)
             for m, kd, psi, e0 in inst]
    ws = mcd.Workspace(sorted(sizes)[-1] + sorted(sizes)[-2])
    Gb, info = mcd.batch_band_green([i[0] for i in inst], [i[1] for i in inst],
                                    [i[2] for i in inst], [i[3] for i in inst], orbs, spins, om,
                                    ws=ws, **kw)
    for a, b in zip(Gb, singles):
        assert np.array_equal(a, b)
    assert ws.stats()["in_use"] == 0
    ws.close()
    tiny = mcd.Workspace(64 << 10)
    with pytest.raises(mcd.McdError) as e:
        mcd.batch_band_green([i[0] for i in inst], [i[1] for i in inst], [i[2] for i in inst],
                             [i[3] for i in inst], orbs, spins, om, ws=tiny, **kw)
    assert e.value.code == mcd.MCD_E_WORKSPACE
    tiny.close()


def test_non_finite_inputs_are_errors_not_nan():
    """A NaN in the start vector or in psi0 is reported as MCD_E_NUMERIC
    (-6) instead of propagating into E0 or G."""
    torch, mcd = require_gpu()
    m, keys = _c1_chain()
    kd = mcd.keys_from_numpy(keys)
    op = mcd.Operator(m, kd, storage="csr")
    phi = torch.from_numpy(W.random_vector(len(keys), 5)).cuda()
    phi[17] = float("nan")
    with pytest.raises(mcd.McdError) as e:
        mcd.lanczos_ground(op, max_iter=50, tol=1e-10, phi0=phi)
    assert e.value.code == -6
    e0, psi, *_ = mcd.lanczos_ground(op, max_iter=400, tol=1e-12, seed=11)
    bad = psi.clone()
    bad[3] = float("nan")
    om = W.matsubara(4, 50.0)
    for wt in (1.0, 0.99):
        with pytest.raises(mcd.McdError) as e:
            mcd.band_lanczos_green(m, kd, bad, e0, [0, 1], [0, 0], om, max_blocks=8, w_t=wt)
        assert e.value.code == -6
    op.close()


def test_degenerate_ground_state_response_is_a_breakdown():
    """H~ = 0 on two states (no bonds, no U, no eps): every state is a
    ground state, (H - E0) vanishes on the complement of psi0 and the
    response solve of the Green-function derivative cannot proceed:
    MCD_E_BREAKDOWN (-7), not a silent partial gradient."""
    torch, mcd = require_gpu()
    m = W.Model(2, [], np.zeros(2), np.zeros(2), 1, 0, "flat")
    keys = fock.sector_keys(2, 1, 0)
    kd = mcd.keys_from_numpy(keys)
    op = mcd.Operator(m, kd, storage="csr")
    e0, psi, *_ = mcd.lanczos_ground(op, max_iter=10, tol=1e-12, seed=3)
    op.close()
    assert e0 == 0.0
    om = W.matsubara(4, 50.0)
    # imaginary weights: with T = 0 the resolvent at i w is imaginary, so a
    # real G_bar would give a zero start-block adjoint and nothing to solve
    gb = 1j * np.ones((4, 1, 1), complex)
    with pytest.raises(mcd.McdError) as e:
        mcd.band_green_vjp(m, kd, psi, e0, [0], [0], om, gb, max_blocks=4)
    assert e.value.code == -7
