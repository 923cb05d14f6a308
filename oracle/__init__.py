"""CPU oracle for Monte Carlo diagonalization (MCD) of the Hubbard model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library: it reads the same seeded inputs (the ``workloads`` module) and
nothing else.

It is plain and slow on purpose: NumPy/SciPy in float64, one step per
paper equation, no blocking or fusion.  Modules and what they follow:

* ``fock``          Fock-state keys, sectors, double occupation (Sec. Model,
                    Sec. Exact diagonalization, the n_U definition).
* ``hamiltonian``   H restricted to a basis, H_mn = <x_m|H|x_n> (Eq.
                    h_matrix_projected) with out-of-basis states discarded
                    (App. Lanczos, last paragraph); plus an independent
                    Jordan-Wigner Kronecker construction used only as a pin.
* ``lanczos``       Lanczos recurrence, Eqs. next_vector / an_bn, and the
                    ground-state reconstruction, Eq. change_basis.
* ``band_lanczos``  band Lanczos with deflation (App. Band Lanczos).
* ``green``         target-weight truncation (Sec. Further truncation),
                    excited subspaces (Eq. excited_subspace), Q matrices and
                    the Lehmann Green function (Eqs. green_qmatrix, q_matrix).
* ``sampler``       the Metropolis chain that draws the truncated basis
                    (variant-1 ratio acceptance, Eq. boltzmann_factor2, with a
                    single random hop per step, variant 2), with a plain-C
                    implementation for large chains.

Parity status of each function is stated in its docstring; a function with
no independent pin says "parity unpinned".
"""
