"""Writes tests/golden/c5_green.json: the oracle's converged ground state and
Green function on the 4x8 t-t' cluster's 50M-state chain basis (the C5
workload at full size), for the GPU test that runs the same pipeline.

Steps, all from the oracle: the basis (oracle.sampler's C chain), H~
(oracle.hamiltonian.build_csr), Lanczos without reorthogonalisation from the
seed-11 start vector to a Ritz residual of 1e-10 relative (the recurrence
without stored vectors), the ground state by a second pass of the same
recurrence (Eq. change_basis), then the Green function of the 16 up-spin
orbitals 0..15 with the target-weight cut w_t = 0.999 (oracle.green: cut,
F~+-, start blocks, band Lanczos with full reorthogonalisation, Lehmann sums)
at 128 Matsubara frequencies (beta = 50).  Stored: E0, the sizes after the
cut, and G at eight of the frequencies.  Runs on the CPU in about an hour and
needs ~25 GB of host memory.

Usage: python tests/golden/make_c5_green.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import green, hamiltonian as ham, lanczos as lz, sampler  # noqa: E402

FREQ_IDX = [0, 1, 2, 3, 7, 15, 31, 127]


def main():
    c = W.config_c5()
    m = c["model"]
    t0 = time.time()
    keys, steps = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                  c["max_steps"])
    print(f"basis {len(keys)} states, {steps} steps, {time.time() - t0:.0f} s", flush=True)
    H = ham.build_csr(keys, m)
    print(f"H~: {H.nnz} stored entries, {time.time() - t0:.0f} s", flush=True)
    phi0 = lz.start_vector(keys, 11)
    r = lz.lanczos_ground(H, phi0, tol=1e-10, max_iter=1000, reorth=False, keep_vectors=False)
    print(f"E0 = {r['e0']!r} after {r['iters']} steps, residual {r['residual']:.3e}, "
          f"{time.time() - t0:.0f} s", flush=True)
    e0, psi = lz.recompute_ground_state(H, phi0, r["alpha"], r["beta"])
    del H
    print(f"psi0 by the second pass, {time.time() - t0:.0f} s", flush=True)
    omega = W.matsubara(128, 50.0)
    G, parts = green.green_mcd(keys, m, psi, e0, list(range(16)), 0, omega, w_t=0.999,
                               return_parts=True)
    print(f"G: kept {len(parts['keys_t'])}, F~+ {len(parts['plus'][2])}, "
          f"F~- {len(parts['minus'][2])}, {time.time() - t0:.0f} s", flush=True)
    out = {"what": "oracle E0 (Lanczos without reorthogonalisation, seed-11 start vector, Ritz "
                   "residual <= 1e-10 relative) and G of the up-spin orbitals 0..15 (w_t = 0.999, "
                   "band Lanczos to exhaustion, Matsubara frequencies (2n+1) pi / 50) on the 4x8 "
                   "periodic t-t' cluster (U=8, (14,14)), 50M-state chain basis (seed 5, burn-in "
                   "1e6, beta_s 0.5)",
           "n": int(len(keys)), "e0": float(e0), "lanczos_iters": int(r["iters"]),
           "residual": float(r["residual"]), "n_keep": int(len(parts["keys_t"])),
           "n_plus": int(len(parts["plus"][2])), "n_minus": int(len(parts["minus"][2])),
           "freq_index": FREQ_IDX, "omega": [float(omega[i]) for i in FREQ_IDX],
           "G_re": [G[i].real.tolist() for i in FREQ_IDX],
           "G_im": [G[i].imag.tolist() for i in FREQ_IDX]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_green.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
