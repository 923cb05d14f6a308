"""Writes tests/golden/c3_green.json: the oracle's Green function of the C3
workload at its full size (2x2 plaquette + 8 baths, U = 8, seed 3, 0.5M
chain states; sites 0..3 of both spins, 64 Matsubara frequencies at beta =
50), against which the GPU forms state their G error.

Steps, all from the oracle: the basis (oracle.sampler's C chain), H~
(oracle.hamiltonian.build_csr), Lanczos without reorthogonalisation from the
seed-11 start vector to a Ritz residual of 1e-12 relative and the ground
state by a second pass of the same recurrence (Eq. change_basis), then per
spin the Green function of sites 0..3 (oracle.green.green_mcd, w_t = 1:
F~+-, start blocks, band Lanczos with full reorthogonalisation up to 480
vectors per sector, Lehmann sums).  G is block diagonal in spin; the two 4x4
blocks are stored for every frequency.  Runs on the CPU in about 15 minutes
and needs ~15 GB of host memory.

Usage: python tests/golden/make_c3_green.py
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

MAX_DIM = 480


def main():
    c = W.config_c3()
    m = c["model"]
    t0 = time.time()
    keys, steps = sampler.chain_c(m, W.neel_start(m), c["seed"], c["n_f"], c["burn_in"],
                                  c["max_steps"])
    H = ham.build_csr(keys, m)
    phi0 = lz.start_vector(keys, 11)
    r = lz.lanczos_ground(H, phi0, tol=1e-12, max_iter=3000, reorth=False, keep_vectors=False)
    e0, psi = lz.recompute_ground_state(H, phi0, r["alpha"], r["beta"])
    print(f"n {len(keys)}, E0 {e0!r}, {r['iters']} steps, residual {r['residual']:.2e}, "
          f"{time.time() - t0:.0f} s", flush=True)
    del H
    om = W.matsubara(64, 50.0)
    blocks, sizes = [], []
    for spin in (0, 1):
        G, parts = green.green_mcd(keys, m, psi, e0, [0, 1, 2, 3], spin, om, max_dim=MAX_DIM,
                                   return_parts=True)
        blocks.append([[[float(v.real), float(v.imag)] for v in row.ravel()] for row in G])
        sizes.append([int(len(parts["plus"][2])), int(len(parts["minus"][2])),
                      int(parts["plus"][3]), int(parts["minus"][3])])
        print(f"spin {spin}: F~+ {sizes[-1][0]}, F~- {sizes[-1][1]}, Krylov {sizes[-1][2]} / "
              f"{sizes[-1][3]}, {time.time() - t0:.0f} s", flush=True)
    out = {"what": "oracle G(i w_n) of sites 0..3 per spin block [spin][freq][4x4 row-major]"
                   "[re, im] on the C3 basis (2x2 plaquette + 8 baths, U=8, seed 3, 0.5M chain "
                   "states); ground state: Lanczos residual 1e-12, second pass; band Lanczos "
                   "with full reorthogonalisation up to 480 vectors per sector",
           "n": int(len(keys)), "chain_steps": int(steps), "e0": float(e0),
           "lanczos_iters": int(r["iters"]), "n_freq": 64, "beta_m": 50.0,
           "sizes_per_spin": sizes, "G": blocks}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_green.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
