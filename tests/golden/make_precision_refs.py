"""Writes tests/golden/precision_refs.json: oracle values against which the
precision of the float32 forms is stated.

* c3: E0 of the 2x2-plaquette + 8-bath impurity model (seed 3) on its
  0.5M-state chain basis, float64 Lanczos to a Ritz residual of 1e-12.
* g20k: E0 and the converged G(i w_n) of the same model family (seed 5) on a
  20,000-state chain basis, 4 impurity sites x 2 spins, the first 16
  Matsubara frequencies at beta = 50; band Lanczos up to 200 block steps of
  the 4 operators of each spin (the result agrees with 100 steps to 2e-13).
  G is block diagonal in spin: the two 4x4 blocks are stored.

Calls the oracle only (basis: oracle.sampler's C chain; H~:
oracle.hamiltonian.build_csr; Lanczos: oracle.lanczos; G: oracle.green).
Runs on the CPU in about a minute.

Usage: python tests/golden/make_precision_refs.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import green as gr, hamiltonian as ham, lanczos as lz, sampler  # noqa: E402

G20K = dict(model_seed=5, chain_seed=4, n_f=20000, burn_in=500, max_steps=10**7, n_freq=16,
            beta_m=50.0, orbitals=[0, 1, 2, 3], max_dim=800)


def main():
    t0 = time.time()
    c = W.config_c3()
    m = c["model"]
    keys, steps = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                  c["max_steps"])
    H = ham.build_csr(keys, m)
    r = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-12, max_iter=3000, reorth=False,
                          keep_vectors=False)
    print(f"c3: n {len(keys)}, E0 {r['e0']!r}, {r['iters']} steps, {time.time() - t0:.0f} s",
          flush=True)
    out = {"c3": {"what": "oracle float64 Lanczos E0 (Ritz residual 1e-12, no "
                          "reorthogonalisation, start vector seed 11) on the C3 chain basis",
                  "n": int(len(keys)), "chain_steps": int(steps), "e0": float(r["e0"]),
                  "iters": int(r["iters"])}}

    g = G20K
    m = W.impurity_plaquette_bath(g["model_seed"])
    keys, _ = sampler.chain_c(m, W.neel_start(m), g["chain_seed"], g["n_f"], g["burn_in"],
                              g["max_steps"])
    H = ham.build_csr(keys, m)
    r = lz.lanczos_ground(H, lz.start_vector(keys, 11), tol=1e-13, max_iter=1000)
    om = W.matsubara(g["n_freq"], g["beta_m"])
    blocks = []
    for spin in (0, 1):
        G = gr.green_mcd(keys, m, r["psi0"], r["e0"], g["orbitals"], spin, om,
                         max_dim=g["max_dim"])
        blocks.append([[[float(v.real), float(v.imag)] for v in row.ravel()] for row in G])
        print(f"g20k: spin {spin} done, {time.time() - t0:.0f} s", flush=True)
    out["g20k"] = dict(g, what="oracle E0 (residual 1e-13) and G(i w_n) per spin block "
                               "[spin][freq][4x4 row-major][re, im]",
                       n=int(len(keys)), e0=float(r["e0"]), G=blocks)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           "precision_refs.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
