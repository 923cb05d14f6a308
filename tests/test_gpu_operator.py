"""GPU parity of the basis and of H~ x (C ABI) against the CPU oracle.

Bit-exact: basis keys, chain step counts, connectivity (row, col) and signed
elements.  Float64 products: max |y - y_ref| <= 1e-12 max |y_ref| (the
summation order differs; each element is a sum of <= 2 n_bonds + 1 terms of
magnitude |t| |x| or |d| |x|, so the rounding difference is a few ulp).
Float32 products: 2e-6 relative (float accumulation of <= 257 terms).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fock, hamiltonian as ham, lanczos as lz, sampler
from tests.gpu_common import log_case, random_model, require_gpu

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


MODELS = {
    "c1": W.config_c1()["model"],
    "ring8_mu4": W.chain(8, U=8.0, mu=4.0, pbc=True),
    "sq3x2_tp": W.square(3, 2, tp=-0.3, U=8.0, pbc=True, n_up=3, n_dn=2),
    "sq2x2_doubled": W.square(2, 2, U=8.0, pbc=True),
    "rand_dup": random_model(7, dup=True),
    "imp": W.impurity_plaquette_bath(3),
}


@pytest.mark.parametrize("name", ["c1", "ring8_mu4", "sq3x2_tp", "rand_dup"])
def test_full_sector_keys(name):
    torch, mcd = require_gpu()
    m = MODELS[name]
    log_case("full_sector_keys", model=name)
    k, _ = mcd.basis_build(m, "full")
    assert np.array_equal(mcd.keys_to_numpy(k), fock.sector_keys(m.n_orb, m.n_up, m.n_dn))


def test_full_sector_keys_edges():
    torch, mcd = require_gpu()
    m = W.chain(12, U=8.0, mu=4.0)
    for nu, nd in ((0, 0), (0, 3), (12, 5), (6, 6)):
        log_case("full_sector_edges", n_up=nu, n_dn=nd)
        k, _ = mcd.basis_build(m, "full", n_up=nu, n_dn=nd)
        assert np.array_equal(mcd.keys_to_numpy(k), fock.sector_keys(12, nu, nd))


def _chain_case(mcd, m, seed, n_f, burn, steps):
    st = W.neel_start(m)
    ko, so = sampler.chain_c(m, st, seed, n_f, burn, steps)
    kg, sg = mcd.basis_build(m, "chain", start_key=st, seed=seed, beta_s=0.5, burn_in=burn,
                             max_steps=steps, n_f=n_f)
    return ko, so, mcd.keys_to_numpy(kg), sg


@pytest.mark.parametrize("case", ["c1", "imp", "c1_short"])
def test_chain_basis_bit_exact(case):
    torch, mcd = require_gpu()
    log_case("chain_basis", case=case)
    if case == "c1":
        c = W.config_c1()
        ko, so, kg, sg = _chain_case(mcd, c["model"], c["seed"], c["n_f"], c["burn_in"],
                                     c["max_steps"])
    elif case == "imp":
        ko, so, kg, sg = _chain_case(mcd, MODELS["imp"], 9, 30000, 1000, 10**7)
    else:   # step cap reached before n_f
        ko, so, kg, sg = _chain_case(mcd, MODELS["c1"], 4, 4900, 10, 2000)
    assert so == sg
    assert np.array_equal(ko, kg)


def test_chain_basis_c2_full_size():
    torch, mcd = require_gpu()
    c = W.config_c2()
    log_case("chain_basis_c2", n_f=c["n_f"])
    ko, so, kg, sg = _chain_case(mcd, c["model"], c["seed"], c["n_f"], c["burn_in"],
                                 c["max_steps"])
    assert len(kg) == c["n_f"] and so == sg and np.array_equal(ko, kg)


def _basis(name, mcd):
    m = MODELS[name]
    if name == "imp":
        keys, _ = sampler.chain_c(m, W.neel_start(m), 9, 20000, 1000, 10**7)
    elif name == "c1":
        c = W.config_c1()
        keys, _ = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                  c["max_steps"])
    else:
        keys = fock.sector_keys(m.n_orb, m.n_up, m.n_dn)
    return m, keys


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("storage", ["csr", "otf"])
def test_connectivity_bit_exact(name, storage):
    torch, mcd = require_gpu()
    m, keys = _basis(name, mcd)
    log_case("connectivity", model=name, storage=storage, n=len(keys))
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
    r, c, v = op.connectivity()
    order = np.lexsort((c, r))
    ro, co, vo = ham.offdiag_pattern(keys, m)
    assert np.array_equal(r[order], ro) and np.array_equal(c[order], co)
    assert np.array_equal(v[order], vo)
    # diagonal
    d = op.diagonal().cpu().numpy()
    assert np.max(np.abs(d - fock.diagonal(keys, m))) <= 1e-13 * max(1.0, np.abs(d).max())
    op.close()


def _kernels(op, storage):
    return op.kernels() if storage == "csr" else [None]


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("storage", ["csr", "otf"])
@pytest.mark.parametrize("nvec", [1, 2, 4, 8, 16])
def test_apply_f64(name, storage, nvec):
    torch, mcd = require_gpu()
    m, keys = _basis(name, mcd)
    log_case("apply_f64", model=name, storage=storage, nvec=nvec, n=len(keys))
    H = ham.build_csr(keys, m)
    x = W.random_vector(len(keys), 100 + nvec, nvec)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
    for kern in _kernels(op, storage) if nvec == 1 else [None]:
        if kern:
            op.set_kernel(kern)
        y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy()
        assert _rel(y, H @ x) <= 1e-12, kern
    op.close()


def test_merge_path_long_and_empty_rows():
    """Merge-path chunking with rows of ~130 nonzeros (fully connected 12-orbital
    model) and with rows that keep no hop at all (sparse subset of a sector)."""
    torch, mcd = require_gpu()
    rng = np.random.default_rng(11)
    amps = [-1.0, -0.5, 0.3, 0.7]          # packed CSR holds <= 32 distinct |t|
    bonds = [(i, j, float(rng.choice(amps))) for i in range(12) for j in range(i + 1, 12)]
    dense = W.Model(12, bonds, rng.uniform(0, 4, 12), rng.uniform(-1, 1, 12), 6, 6, "dense")
    full = fock.sector_keys(12, 6, 6)
    cases = {"dense_full": (dense, full[:60000]),
             "sparse_subset": (W.chain(12, U=8.0, mu=4.0), np.sort(rng.choice(full, 30000, replace=False))),
             "mixed": (dense, np.sort(np.concatenate([full[:3000], rng.choice(full[3000:], 20000, replace=False)])))}
    for name, (m, keys) in cases.items():
        log_case("merge_rows", case=name, n=len(keys))
        H = ham.build_csr(keys, m)
        x = W.random_vector(len(keys), 3)
        op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
        for kern in op.kernels():
            op.set_kernel(kern)
            y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy()
            assert _rel(y, H @ x) <= 1e-12, (name, kern)
            y32 = op.apply(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
            assert _rel(y32.astype(np.float64), H @ x) <= 2e-6, (name, kern)
        op.close()


def test_block_product_tiles():
    """Block products in one-pass row tiles: rows of ~48 nonzeros (the first
    40,000 states of a fully connected 12-orbital model's sector) give
    64-row blocks of <= 4096 and 128-row blocks of <= 8192 nonzeros, so one
    or two lanes per row (float32 x 4 / x 8, float64 x 2 / x 4) take the
    large 128-row tiles and four or eight lanes the 4096-word ones; a sparse
    chain subset takes full tiles.  Against the whole-matrix product, and
    the shared columns of different block widths bit for bit (the
    per-column sum is the same whatever the tile)."""
    torch, mcd = require_gpu()
    rng = np.random.default_rng(5)
    amps = [-1.0, -0.5, 0.3, 0.7]
    bonds = [(i, j, float(rng.choice(amps))) for i in range(12) for j in range(i + 1, 12)]
    dense = W.Model(12, bonds, rng.uniform(0, 4, 12), rng.uniform(-1, 1, 12), 6, 6, "dense")
    full = fock.sector_keys(12, 6, 6)
    cases = {"dense": (dense, full[:40000], (64, 128)),
             "chain": (W.chain(12, U=8.0, mu=4.0), np.sort(rng.choice(full, 30000, replace=False)), None)}
    for name, (m, keys, rpb) in cases.items():
        H = ham.build_csr(keys, m)
        op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
        info = op.info()
        log_case("block_tiles", case=name, n=len(keys), rows_per_block=info["rows_per_block"],
                 rows_per_block_l=info["rows_per_block_l"])
        if rpb is not None:
            assert (info["rows_per_block"], info["rows_per_block_l"]) == rpb
        for dt, tdt, tol in ((np.float64, torch.float64, 1e-12), (np.float32, torch.float32, 2e-6)):
            X = W.random_vector(len(keys), 9, 16).astype(dt)
            Xd = torch.from_numpy(X).cuda()
            Y = {}
            for nv in (2, 4, 8, 16):
                Y[nv] = op.apply(Xd[:, :nv].contiguous()).cpu().numpy()
                ref = H @ X[:, :nv].astype(np.float64)
                assert _rel(Y[nv].astype(np.float64), ref) <= tol, (name, dt, nv)
            for nv in (2, 4, 8):
                assert np.array_equal(Y[16][:, :nv], Y[nv]), (name, dt, nv)
        op.close()


@pytest.mark.parametrize("storage", ["csr", "otf"])
@pytest.mark.parametrize("nvec", [1, 8, 16])
def test_apply_f32(storage, nvec):
    torch, mcd = require_gpu()
    m, keys = _basis("imp", mcd)
    log_case("apply_f32", storage=storage, nvec=nvec)
    H = ham.build_csr(keys, m)
    x = W.random_vector(len(keys), 7, nvec).astype(np.float32)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
    y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    assert _rel(y, H @ x.astype(np.float64)) <= 2e-6


def test_apply_edges():
    """Ragged and degenerate bases: 1 state, 2 states, no kept hops, sizes that
    end mid-block, and a basis mixing two sectors (block diagonal)."""
    torch, mcd = require_gpu()
    m = MODELS["sq3x2_tp"]
    full = fock.sector_keys(6, 3, 2)
    rng = np.random.default_rng(3)
    other = fock.sector_keys(6, 2, 2)
    cases = {
        "one": full[:1], "two": full[[0, -1]],
        "ragged": np.sort(rng.choice(full, 257, replace=False)),
        "ragged2": np.sort(rng.choice(full, 131, replace=False)),
        "two_sectors": np.union1d(full[::2], other[::3]),
    }
    for name, keys in cases.items():
        for storage in ("csr", "otf"):
            log_case("apply_edges", case=name, storage=storage, n=len(keys))
            H = ham.build_csr(keys, m)
            x = W.random_vector(len(keys), 1)
            op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage=storage)
            for kern in _kernels(op, storage):
                if kern:
                    op.set_kernel(kern)
                y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy()
                assert _rel(y, H @ x) <= 1e-12, (name, kern)
            op.close()


def test_invalid_keys_rejected():
    torch, mcd = require_gpu()
    m = MODELS["sq3x2_tp"]
    full = fock.sector_keys(6, 3, 2)
    bad = full[::-1].copy()
    with pytest.raises(mcd.McdError):
        mcd.Operator(m, mcd.keys_from_numpy(bad))
    dup = np.concatenate([full[:5], full[4:6]])
    with pytest.raises(mcd.McdError):
        mcd.Operator(m, mcd.keys_from_numpy(dup))


def test_apply_c2_full_size_sampled_rows():
    """C2 at its full size (4x4 t-t', 4M chain states): every row of the GPU
    product is produced by the timed kernel; 3000 seeded rows are checked
    against the oracle's element definition, plus H = H^T via <x|Hy> = <Hx|y>."""
    torch, mcd = require_gpu()
    c = W.config_c2()
    m = c["model"]
    keys, _ = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                              c["max_steps"])
    log_case("apply_c2", n=len(keys))
    x = W.random_vector(len(keys), 21)
    rows = np.sort(np.random.default_rng(5).choice(len(keys), 3000, replace=False))
    ref = ham.apply_rows(keys, rows, m, x)
    kd = mcd.keys_from_numpy(keys)
    y_stream = None
    for storage, kern in (("csr", "stream"), ("csr", "merge"), ("csr", "stream_xcd"),
                          ("csr", "rowchunk"), ("csr", "stream_small"),
                          ("csr", "stream_small_xcd"), ("csr", "grouped"),
                          ("csr", "grouped_xcd"), ("otf", None)):
        op = mcd.Operator(m, kd, storage=storage)
        if kern:
            op.set_kernel(kern)
        xt = torch.from_numpy(x).cuda()
        y = op.apply(xt)
        assert _rel(y.cpu().numpy()[rows], ref) <= 1e-12
        if kern == "stream":
            y_stream = y.clone()
        if kern not in (None, "stream", "merge", "rowchunk"):
            # same terms in the same order per row: bit-identical to row-major
            # (the merge path splits long rows and adds the pieces in a fix-up;
            # the row-chunk kernel sums a row's chunks in another association)
            assert torch.equal(y, y_stream), kern
        x2 = torch.from_numpy(W.random_vector(len(keys), 22)).cuda()
        y2 = op.apply(x2)
        a, b = float(torch.dot(x2, y)), float(torch.dot(xt, y2))
        assert abs(a - b) <= 1e-11 * max(abs(a), 1.0)
        if storage == "csr":
            info = op.info()
            assert info["nnz"] > 0
            print("[c2] nnz", info["nnz"], "rows/block", info["rows_per_block"], flush=True)
        op.close()


def test_c5_full_size_keys_and_sampled_rows():
    """The 4x8 t-t' cluster at its full size (50M chain states): GPU chain keys
    bit-exact with the oracle's chain; float64 products (the kernel the
    operator tunes to, as timed) and float32 16-vector block products on
    20000 seeded rows against the oracle's element definition; on-the-fly
    float64 too."""
    torch, mcd = require_gpu()
    c = W.config_c5()
    m = c["model"]
    log_case("c5_keys", n_f=c["n_f"])
    kd, steps = mcd.basis_build(m, "chain", start_key=W.neel_start(m), seed=c["seed"],
                                beta_s=c["beta_s"], burn_in=c["burn_in"],
                                max_steps=c["max_steps"], n_f=c["n_f"])
    keys, steps_ref = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                      c["max_steps"])
    got = mcd.keys_to_numpy(kd)
    assert len(got) == len(keys) == c["n_f"] and steps == steps_ref
    assert np.array_equal(got, keys)
    n = len(keys)
    rows = np.sort(np.random.default_rng(9).choice(n, 20000, replace=False))
    x = W.random_vector(n, 31)
    ref = ham.apply_rows(keys, rows, m, x)
    log_case("c5_apply_f64_csr", n=n)
    op = mcd.Operator(m, kd, storage="csr")
    y = op.apply(torch.from_numpy(x).cuda())
    assert _rel(y.cpu().numpy()[rows], ref) <= 1e-12
    X = W.random_vector(n, 32, nvec=16, dtype=np.float32)
    refX = ham.apply_rows(keys, rows, m, X.astype(np.float64))
    log_case("c5_apply_f32_b16_csr", n=n)
    Y = op.apply(torch.from_numpy(X).cuda())
    assert _rel(Y.cpu().numpy()[rows].astype(np.float64), refX) <= 2e-6
    op.close()
    del Y
    log_case("c5_apply_f64_otf", n=n)
    op = mcd.Operator(m, kd, storage="otf")
    y = op.apply(torch.from_numpy(x).cuda())
    assert _rel(y.cpu().numpy()[rows], ref) <= 1e-12
    op.close()


@pytest.mark.parametrize("case", ["c1", "ring4_18", "imp", "c1_beta0_full", "sq4x4_tp"])
def test_step_sampler_bit_exact(case):
    """The paper's step sampler on the GPU against the oracle (keys, steps)."""
    torch, mcd = require_gpu()
    m, nf, beta, seed = {"c1": (W.config_c1()["model"], 2000, 0.2, 7),
                         "ring4_18": (W.chain(4, U=8.0, mu=4.0), 18, 0.2, 3),
                         "imp": (W.impurity_plaquette_bath(3), 5000, 0.2, 7),
                         "c1_beta0_full": (W.config_c1()["model"], 4900, 0.0, 1),
                         "sq4x4_tp": (W.config_c2()["model"], 60000, 0.2, 5)}[case]
    log_case("step_sampler", case=case, n_f=nf)
    st = W.neel_start(m)
    ko, so = sampler.bfs_numpy(m, st, seed, beta, nf, 1000)
    kg, sg = mcd.basis_build(m, "steps", start_key=st, seed=seed, beta_s=beta, max_steps=1000,
                             n_f=nf)
    assert so == sg and np.array_equal(ko, mcd.keys_to_numpy(kg))


@pytest.mark.parametrize("case", ["ring8_l1", "ring8_l2", "ring8_l2_cut", "c1_l1", "sq4x4_l1",
                                  "ring12_l2"])
def test_step_sampler_preaccepted_levels_bit_exact(case):
    """Pre-accepted low-n_U levels (enumerated on the GPU by ranked
    combinations) then the step search, against the oracle's brute-force
    level sets; 'cut': the levels alone exceed N_f (no step is taken)."""
    torch, mcd = require_gpu()
    m, nf, lvl = {"ring8_l1": (W.chain(8, U=8.0, mu=4.0), 600, 1),
                  "ring8_l2": (W.chain(8, U=8.0, mu=4.0), 2500, 2),
                  "ring8_l2_cut": (W.chain(8, U=8.0, mu=4.0), 1000, 2),
                  "c1_l1": (W.config_c1()["model"], 3000, 1),
                  "sq4x4_l1": (W.square(4, 4, U=8.0, mu=4.0, pbc=True, n_up=7, n_dn=7), 200000, 1),
                  "ring12_l2": (W.chain(12, U=8.0, mu=4.0), 100000, 2)}[case]
    log_case("step_sampler_pre", case=case, n_f=nf, level=lvl)
    st = W.neel_start(m)
    ko, so = sampler.bfs_numpy(m, st, 5, 0.2, nf, 1000, pre_level=lvl)
    kg, sg = mcd.basis_build(m, "steps", start_key=st, seed=5, beta_s=0.2, max_steps=1000,
                             n_f=nf, pre_level=lvl)
    assert so == sg and np.array_equal(ko, mcd.keys_to_numpy(kg))


def _grouped_cases():
    rng = np.random.default_rng(17)
    ch12 = W.chain(12, U=8.0, mu=4.0, pbc=True, n_up=6, n_dn=6)
    full12 = fock.sector_keys(12, 6, 6)
    c1 = W.config_c1()
    m1 = c1["model"]
    k1, _ = sampler.chain_c(m1, W.neel_start(m1), c1["seed"], c1["n_f"], c1["burn_in"],
                            c1["max_steps"])
    return {
        # one up-string segment of 924 rows spans several blocks
        "chain12_full": (ch12, full12, True),
        # 30% of the sector: short rows, chunks split by the 256-row cap
        "chain12_subset": (ch12, np.sort(rng.choice(full12, 250000, replace=False)), True),
        # C1 full sector: 70 segments of 70 rows, several segments per block
        "c1_full": (m1, fock.sector_keys(8, 4, 4), True),
        # C1 chain basis (2000 states, ~28 rows per segment): built or not
        "c1_chain": (m1, k1, None),
        # segments of ~1 row: the layout is not built
        "sparse": (ch12, np.sort(rng.choice(full12, 900, replace=False)), False),
    }


@pytest.mark.parametrize("case", ["chain12_full", "chain12_subset", "c1_full", "c1_chain", "sparse"])
def test_grouped_layout(case):
    """Kernels 7 / 8 (grouped entry order) against the oracle and bit-for-bit
    against the row-major kernel, float64 and float32; the fused scale + dot
    of the Lanczos step through the grouped kernels gives the oracle's E0."""
    torch, mcd = require_gpu()
    m, keys, expect = _grouped_cases()[case]
    log_case("grouped", case=case, n=len(keys))
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
    have = op.info()["grouped_blocks"] > 0
    print(f"[grouped] {case}: n {len(keys)} blocks {op.info()['grouped_blocks']} "
          f"chosen {op.info()['kernel']}", flush=True)
    if expect is not None:
        assert have == expect
    if not have:
        with pytest.raises(mcd.McdError):
            op.set_kernel("grouped")
        op.close()
        return
    H = ham.build_csr(keys, m)
    x = W.random_vector(len(keys), 5)
    xt = torch.from_numpy(x).cuda()
    x32 = torch.from_numpy(x.astype(np.float32)).cuda()
    op.set_kernel("stream")
    y_ref, y32_ref = op.apply(xt), op.apply(x32)
    for kern in ("grouped", "grouped_xcd"):
        op.set_kernel(kern)
        y = op.apply(xt)
        assert _rel(y.cpu().numpy(), H @ x) <= 1e-12, kern
        assert torch.equal(y, y_ref), kern
        assert torch.equal(op.apply(x32), y32_ref), kern
    if len(keys) > 300000:
        op.close()
        return
    ro = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13)
    for kern in ("grouped", "grouped_xcd"):
        op.set_kernel(kern)
        e0, psi, *_ = mcd.lanczos_ground(op, max_iter=400, tol=1e-12, seed=11)
        assert abs(e0 - ro["e0"]) <= 1e-10 * abs(ro["e0"]), kern
    op.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_block_product_alignment_paths(dtype):
    """Blocks whose rows are whole 16-byte pieces and 16-byte aligned take the
    16-byte-gather kernel, misaligned ones the one-value-per-lane kernel: both
    add the same terms in the same order (bit-identical), and match the
    oracle's CSR product."""
    torch, mcd = require_gpu()
    m, keys = _basis("imp", mcd)
    n = len(keys)
    log_case("block_alignment", dtype=dtype, n=n)
    op = mcd.Operator(m, mcd.keys_from_numpy(keys), storage="csr")
    H = ham.build_csr(keys, m)
    tdt, code, es = (torch.float32, 1, 4) if dtype == "f32" else (torch.float64, 0, 8)
    for nvec in (2, 4, 8, 16):
        x = W.random_vector(n, 40 + nvec, nvec)
        xa = torch.from_numpy(x).to(tdt).cuda()
        ya = op.apply(xa)
        bx = torch.zeros(n * nvec + 4, dtype=tdt, device="cuda")
        by = torch.zeros(n * nvec + 4, dtype=tdt, device="cuda")
        bx[1:1 + n * nvec] = xa.reshape(-1)
        assert op.apply_raw(code, nvec, bx.data_ptr() + es, by.data_ptr() + es) == 0
        torch.cuda.synchronize()
        ym = by[1:1 + n * nvec].reshape(n, nvec)
        assert torch.equal(ym, ya), nvec
        ref = H @ xa.double().cpu().numpy()
        tol = 2e-6 if dtype == "f32" else 1e-12
        assert _rel(ya.double().cpu().numpy(), ref) <= tol, nvec
    op.close()
