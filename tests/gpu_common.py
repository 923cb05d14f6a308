"""Shared helpers of the GPU parity tests (inputs only; no arithmetic)."""
import numpy as np
import pytest

import workloads as W


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_22975_amd as mcd     # raises if libmcd.so is missing
    mcd.lib()
    return torch, mcd


def random_model(seed, n=6, n_up=3, n_dn=2, dup=False):
    rng = np.random.default_rng(seed)
    bonds = [(int(i), int(j), float(rng.normal())) for i in range(n) for j in range(i + 1, n)
             if rng.uniform() < 0.6]
    if dup and bonds:
        bonds.append((bonds[0][1], bonds[0][0], 0.25))     # same pair, reversed: amplitudes add
    return W.Model(n, bonds, rng.uniform(0, 8, n), rng.uniform(-2, 2, n), n_up, n_dn, "rand")


def log_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
