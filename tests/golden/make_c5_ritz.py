"""Writes tests/golden/c5_ritz200.json: the oracle's Lanczos Ritz value after
200 steps (no reorthogonalisation, start vector of seed 11) on the 4x8 t-t'
cluster's 50M-state chain basis, for the GPU test that checks the same
200-step value at full size.  Calls the oracle only (basis: oracle.sampler's
C chain; H~: oracle.hamiltonian.build_csr; Lanczos: oracle.lanczos).  Runs
on the CPU in about half an hour and needs ~20 GB of host memory.

Usage: python tests/golden/make_c5_ritz.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import hamiltonian as ham, lanczos as lz, sampler  # noqa: E402


def main():
    c = W.config_c5()
    m = c["model"]
    t0 = time.time()
    keys, steps = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                  c["max_steps"])
    print(f"basis {len(keys)} states, {steps} steps, {time.time() - t0:.0f} s", flush=True)
    H = ham.build_csr(keys, m)
    print(f"H~: {H.nnz} stored entries, {time.time() - t0:.0f} s", flush=True)
    r = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=0.0, max_iter=200, reorth=False,
                          keep_vectors=False)
    print(f"E0(200) = {r['e0']!r}, {time.time() - t0:.0f} s", flush=True)
    out = {"what": "oracle Lanczos Ritz value after 200 steps, no reorthogonalisation, start "
                   "vector seed 11, on the 4x8 periodic t-t' cluster (U=8, (14,14)), 50M-state "
                   "chain basis (seed 5, burn-in 1e6, beta_s 0.5)",
           "n": int(len(keys)), "chain_steps": int(steps), "nnz_stored": int(H.nnz),
           "e0_200": float(r["e0"]), "alpha_0": float(r["alpha"][0])}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_ritz200.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
