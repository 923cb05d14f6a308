"""GPU parity of mcd_band_lanczos_green (w_t cut, F~+-, start blocks, block
Lanczos, resolvent) against the oracle's band Lanczos + Lehmann sums.

Same Krylov space on both sides: the GPU's block step adds P = padded p
directions, the oracle's band method one at a time, so max_dim = p * blocks
per spin sector gives the same projected resolvent.  Float64 tolerance:
1e-9 max |G| (both sides reorthogonalise fully; the resolvent at Matsubara
frequencies is well conditioned, |z - E| >= pi/beta).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fock, green as gr, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, require_gpu

pytestmark = pytest.mark.gpu
OM = W.matsubara(64, 50.0)


def _gs(m, keys):
    H = ham.build_csr(keys, m)
    r = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13)
    return r["e0"], r["psi0"]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _oracle_G(keys, m, psi, e0, orbs, spins, blocks, w_t=1.0):
    """Oracle G for a selection that may mix spins: per-spin band runs."""
    p = len(orbs)
    G = np.zeros((len(OM), p, p), complex)
    for s in (0, 1):
        sel = [q for q in range(p) if spins[q] == s]
        if not sel:
            continue
        o = [orbs[q] for q in sel]
        Gs = gr.green_mcd(keys, m, psi, e0, o, s, OM, max_dim=len(o) * blocks, w_t=w_t)
        for i, qi in enumerate(sel):
            for j, qj in enumerate(sel):
                G[:, qi, qj] = Gs[:, i, j]
    return G


def _c1_chain():
    c = W.config_c1()
    m = c["model"]
    k, _ = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"], c["max_steps"])
    return m, k


@pytest.mark.parametrize("sel", ["up4", "mixed8", "ragged3", "all16"])
def test_green_c1_chain_vs_oracle(sel):
    torch, mcd = require_gpu()
    m, keys = _c1_chain()
    orbs, spins = {"up4": ([0, 1, 2, 3], [0] * 4), "mixed8": ([0, 1, 2, 3] * 2, [0] * 4 + [1] * 4),
                   "ragged3": ([1, 5, 6], [1, 0, 1]),
                   "all16": (list(range(8)) * 2, [0] * 8 + [1] * 8)}[sel]
    log_case("green_c1", sel=sel)
    e0, psi = _gs(m, keys)
    blocks = 30
    Go = _oracle_G(keys, m, psi, e0, orbs, spins, blocks)
    G, info = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                     e0, orbs, spins, OM, max_blocks=blocks)
    assert _rel(G, Go) <= 1e-9
    # unbatched reference form: one single-vector product per block column
    Gc, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                   e0, orbs, spins, OM, max_blocks=blocks, per_column=True)
    assert _rel(Gc, G) <= 1e-11
    # three-term block recurrence only (no reorthogonalisation), float64
    G0, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                   e0, orbs, spins, OM, max_blocks=blocks, reorth=0)
    err0 = _rel(G0, Go)
    print("[green] reorth=0 rel err", err0, flush=True)
    assert err0 <= 1e-7


def test_green_p16_one_sector_vs_oracle():
    """p = 16 in one spin sector -- the 16 up orbitals of a 16-site ring (U = 8,
    mu = 4, half filling) on a 5,000-state chain basis -- against the
    oracle's band Lanczos G on the same basis: float64 blocks with two
    reorthogonalisation passes to 1e-9 of max |G|, float32 blocks with one
    pass to 1e-4.  This reaches the P = 16 partial Gram matrices (matrix-core
    form) of both block precisions on excited sectors whose row counts end
    inside a row group."""
    torch, mcd = require_gpu()
    m = W.chain(16, t=1.0, U=8.0, mu=4.0, pbc=True)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 7, 5000, 1000, 10**8)
    log_case("green_p16", n=len(keys))
    e0, psi = _gs(m, keys)
    orbs, spins = list(range(16)), [0] * 16
    blocks = 8
    Go = _oracle_G(keys, m, psi, e0, orbs, spins, blocks)
    for prec, reorth, tol in (("f64", 2, 1e-9), ("f32", 1, 1e-4)):
        G, info = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys),
                                         torch.from_numpy(psi).cuda(), e0, orbs, spins, OM,
                                         max_blocks=blocks, precision=prec, reorth=reorth)
        err = _rel(G, Go)
        print(f"[green p16] {prec} reorth={reorth} rel err {err:.2e} "
              f"(n+ {info.n_plus}, n- {info.n_minus})", flush=True)
        assert info.n_plus % 16 != 0 or info.n_minus % 16 != 0
        assert err <= tol


def test_green_exhausted_equals_dense_definition():
    """Small space run to exhaustion: G equals the dense Lehmann sum over the
    truncated H~+- (the definition, Eqs. green_plus / green_minus)."""
    torch, mcd = require_gpu()
    m = W.chain(6, U=6.0, mu=3.0, pbc=True, n_up=3, n_dn=3)
    keys = fock.sector_keys(6, 3, 3)
    e0, psi = _gs(m, keys)
    orbs, spins = [0, 1, 2, 4], [0, 0, 0, 0]
    Gd = gr.green_dense(m, keys, psi[:, None], e0, orbs, 0, 1j * OM)
    G, info = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                     e0, orbs, spins, OM, max_blocks=200)
    assert _rel(G, Gd) <= 1e-9


def test_green_free_fermions_closed_form():
    torch, mcd = require_gpu()
    m = W.chain(6, U=0.0, pbc=True, n_up=3, n_dn=3)
    keys = fock.sector_keys(6, 3, 3)
    e0, psi = _gs(m, keys)
    h = np.zeros((6, 6))
    for i, j, t in m.bonds:
        h[i, j] += t
        h[j, i] += t
    G0 = np.array([np.linalg.inv(1j * w * np.eye(6) - h) for w in OM])
    G, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                  e0, list(range(6)), [1] * 6, OM, max_blocks=100)
    assert np.max(np.abs(G - G0)) <= 1e-10


def test_green_wt_truncation_vs_oracle():
    torch, mcd = require_gpu()
    m = W.config_c1()["model"]
    keys = fock.sector_keys(8, 4, 4)
    e0, psi = _gs(m, keys)
    orbs, spins = [0, 2, 5], [0, 0, 0]
    for wt in (0.9, 0.99):
        log_case("green_wt", w_t=wt)
        k2, _ = gr.truncate_wt(keys, psi, wt)
        Go = _oracle_G(keys, m, psi, e0, orbs, spins, 25, w_t=wt)
        G, info = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys),
                                         torch.from_numpy(psi).cuda(), e0, orbs, spins, OM,
                                         max_blocks=25, w_t=wt)
        assert info.n_truncated == len(k2)
        assert _rel(G, Go) <= 1e-9


def test_green_impurity_p8_and_sum_rule():
    """C3-shaped impurity model (2x2 + 8 baths, U = 8), chain basis, p = 8."""
    torch, mcd = require_gpu()
    m = W.impurity_plaquette_bath(3)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 9, 20000, 1000, 10**7)
    e0, psi = _gs(m, keys)
    orbs, spins = [0, 1, 2, 3] * 2, [0] * 4 + [1] * 4
    blocks = 20
    Go = _oracle_G(keys, m, psi, e0, orbs, spins, blocks)
    G, info = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                     e0, orbs, spins, OM, max_blocks=blocks)
    assert _rel(G, Go) <= 1e-9
    # tail: i w G(i w) -> identity
    Gt, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                   e0, orbs, spins, np.array([1e7]), max_blocks=blocks)
    assert np.max(np.abs(1j * 1e7 * Gt[0] - np.eye(8))) < 1e-5
    # float32 Krylov blocks, float64 recurrence
    G32, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                    e0, orbs, spins, OM, max_blocks=blocks, precision="f32")
    err = _rel(G32, Go)
    print("[green] f32 rel err", err, flush=True)
    assert err <= 1e-4


def test_green_empty_excited_sectors():
    """Degenerate excited sectors: with every up orbital occupied (n_up =
    n_orb) no c+_up image exists, so F~+ of the up-spin selection is empty and
    G_up = G- only; with no down electron F~- of the down-spin selection is
    empty and G_dn = G+ only.  Against the oracle's dense Lehmann sums over
    the full sectors (which skip an empty sector), and the sum rule of the
    surviving part (G -> 1/(i w) at large w: the start block keeps its
    weight)."""
    torch, mcd = require_gpu()
    base = W.chain(6, U=4.0, mu=2.0, pbc=True)
    for n_up, n_dn, orbs, spins in ((6, 3, [0, 2, 5], [0, 0, 0]), (3, 0, [1, 4], [1, 1]),
                                    (6, 0, [0, 3, 1], [0, 0, 1])):
        m = base.with_sector(n_up, n_dn)
        keys = fock.sector_keys(6, n_up, n_dn)
        log_case("green_empty_sector", n_up=n_up, n_dn=n_dn, n=len(keys))
        e0, psi = _gs(m, keys)
        G, gi = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(),
                                       e0, orbs, spins, OM, max_blocks=40)
        ref = np.zeros_like(G)
        for s in (0, 1):
            sel = [q for q in range(len(orbs)) if spins[q] == s]
            if not sel:
                continue
            Gs = gr.green_exact(keys, m, psi, e0, [orbs[q] for q in sel], s, OM)
            for i, qi in enumerate(sel):
                for j, qj in enumerate(sel):
                    ref[:, qi, qj] = Gs[:, i, j]
        assert _rel(G, ref) <= 1e-9, (n_up, n_dn)
        big = 1e6
        Gt, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys),
                                       torch.from_numpy(psi).cuda(), e0, orbs, spins,
                                       np.array([big]), max_blocks=40)
        assert np.allclose(Gt[0] * 1j * big, np.eye(len(orbs)), atol=1e-5), (n_up, n_dn)


def test_green_deflation_duplicate_selection():
    torch, mcd = require_gpu()
    m, keys = _c1_chain()
    e0, psi = _gs(m, keys)
    G, _ = mcd.band_lanczos_green(m, mcd.keys_from_numpy(keys), torch.from_numpy(psi).cuda(), e0,
                                  [0, 0, 3], [0, 0, 0], OM, max_blocks=20)
    Go = _oracle_G(keys, m, psi, e0, [0, 3], [0, 0], 20)
    assert _rel(G[:, 0, 0], G[:, 1, 1]) < 1e-10
    assert _rel(G[:, 0, 2], Go[:, 0, 1]) < 1e-8


def test_green_stops_at_convergence():
    """g_tol: the band runs stop once G at the check points has settled; the
    result agrees with a run 48 block steps longer to well within g_tol, and
    the same g_tol gives the same stopping point in float64 every time."""
    torch, mcd = require_gpu()
    m = W.impurity_plaquette_bath(5)
    keys, _ = sampler.chain_c(m, W.neel_start(m), 4, 20000, 500, 10**7)
    log_case("green_gtol", n=len(keys))
    e0, psi = _gs(m, keys)
    kd = mcd.keys_from_numpy(keys)
    pt = torch.from_numpy(psi).cuda()
    orbs, spins = [0, 1, 2, 3, 0, 1, 2, 3], [0, 0, 0, 0, 1, 1, 1, 1]
    om = W.matsubara(32, 50.0)
    G1, i1 = mcd.band_lanczos_green(m, kd, pt, e0, orbs, spins, om, max_blocks=300, reorth=2,
                                    g_tol=1e-9)
    assert i1.iters < 300
    G2, i2 = mcd.band_lanczos_green(m, kd, pt, e0, orbs, spins, om, max_blocks=i1.iters + 48,
                                    reorth=2)
    assert _rel(G1, G2) <= 1e-8
    G3, i3 = mcd.band_lanczos_green(m, kd, pt, e0, orbs, spins, om, max_blocks=300, reorth=2,
                                    g_tol=1e-9)
    assert i3.iters == i1.iters and np.array_equal(G1, G3)


def test_c5_full_size_e0_and_green():
    """C5 at its full size (4x8 t-t', 50M chain states), end to end on the GPU
    against the oracle's own run of the same pipeline
    (tests/golden/c5_green.json, written by tests/golden/make_c5_green.py from
    the oracle alone): float64 Lanczos from the seed-11 start vector to a
    1e-10 Ritz residual, E0 to 1e-10 relative; the w_t = 0.999 cut and F~+-
    (sizes equal); G of the up-spin orbitals 0..15 (band Lanczos to
    exhaustion) at eight Matsubara frequencies to 1e-7 of max |G| (both
    ground states carry a residual of ~1e-10 |E0|, which G sees linearly)."""
    import json
    import os
    torch, mcd = require_gpu()
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_green.json")))
    c = W.config_c5()
    m = c["model"]
    log_case("green_c5", n_f=c["n_f"])
    kd, _ = mcd.basis_build(m, "chain", start_key=W.neel_start(m), seed=c["seed"],
                            beta_s=c["beta_s"], burn_in=c["burn_in"], max_steps=c["max_steps"],
                            n_f=c["n_f"])
    assert kd.numel() == gold["n"]
    op = mcd.Operator(m, kd, storage="csr")
    e0, psi, _, _, info = mcd.lanczos_ground(op, max_iter=1000, tol=1e-10, seed=11,
                                             store_vectors=False)
    op.close()
    print("[c5] E0 gpu", e0, "oracle", gold["e0"], "iters", info.iters, gold["lanczos_iters"],
          flush=True)
    assert info.converged
    assert abs(e0 - gold["e0"]) <= 1e-10 * abs(gold["e0"])
    om = W.matsubara(128, 50.0)
    G, gi = mcd.band_lanczos_green(m, kd, psi, e0, list(range(16)), [0] * 16, om,
                                   max_blocks=200, precision="f64", w_t=0.999, reorth=2)
    assert (gi.n_truncated, gi.n_plus, gi.n_minus) == (gold["n_keep"], gold["n_plus"],
                                                       gold["n_minus"])
    ref = np.array(gold["G_re"]) + 1j * np.array(gold["G_im"])
    got = G[gold["freq_index"]]
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    print("[c5] G max rel diff", err, flush=True)
    assert err <= 1e-7


def test_c3_full_size_green_vs_oracle():
    """C3 at its full size (2x2 plaquette + 8 baths, 0.5M chain states, sites
    0..3 of both spins, 64 Matsubara frequencies) against the oracle's G of
    the same basis (tests/golden/c3_green.json, written by
    tests/golden/make_c3_green.py from the oracle alone; oracle ground state
    at a 1e-12 residual, band Lanczos with full reorthogonalisation): the
    float64 form (two reorthogonalisation passes, run until G settles to
    1e-10) to 1e-9 of max |G| (6e-14 seen), the float32-block form to 1e-5
    (2e-6 seen); G is block diagonal in spin."""
    import json
    import os
    torch, mcd = require_gpu()
    go = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_green.json")))
    c = W.config_c3()
    m = c["model"]
    log_case("green_c3", n_f=c["n_f"])
    kd, _ = mcd.basis_build(m, "chain", start_key=W.neel_start(m), seed=c["seed"],
                            beta_s=c["beta_s"], burn_in=c["burn_in"], max_steps=c["max_steps"],
                            n_f=c["n_f"])
    assert kd.numel() == go["n"]
    op = mcd.Operator(m, kd, storage="csr")
    e0, psi, _, _, info = mcd.lanczos_ground(op, max_iter=3000, tol=1e-12, seed=11)
    op.close()
    assert info.converged and abs(e0 - go["e0"]) <= 1e-11 * abs(go["e0"])
    om = W.matsubara(go["n_freq"], go["beta_m"])
    ref = np.zeros((len(om), 8, 8), dtype=np.complex128)
    for sp in (0, 1):
        b = np.array(go["G"][sp])
        ref[:, 4 * sp:4 * sp + 4, 4 * sp:4 * sp + 4] = (b[:, :, 0] + 1j * b[:, :, 1]).reshape(
            len(om), 4, 4)
    orbs, spins = [0, 1, 2, 3] * 2, [0] * 4 + [1] * 4
    for prec, reorth, gt, tol in (("f64", 2, 1e-10, 1e-9), ("f32", 0, 1e-6, 1e-5)):
        G, gi = mcd.band_lanczos_green(m, kd, psi, e0, orbs, spins, om, max_blocks=200,
                                       precision=prec, reorth=reorth, g_tol=gt)
        err = float(np.abs(G - ref).max() / np.abs(ref).max())
        print(f"[c3] {prec}: {gi.iters} block steps, G max rel diff {err:.2e}", flush=True)
        assert err <= tol, prec
