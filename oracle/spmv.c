/* Plain-C product y = A x of a float64 CSR matrix (row pointers int64,
 * columns int32), rows split over the host cores with OpenMP: the oracle's
 * all-core timing of H~ x (A from oracle.hamiltonian, the definition
 * H~_mn = <x_m|H|x_n> of Eq. h_matrix_projected).  Test infrastructure only.
 */
#include <stdint.h>
#include <omp.h>

void csr_matvec(int64_t nrows, const int64_t *indptr, const int32_t *indices,
                const double *data, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; r++) {
        double s = 0.0;
        for (int64_t k = indptr[r]; k < indptr[r + 1]; k++) s += data[k] * x[indices[k]];
        y[r] = s;
    }
}

int csr_threads(void) { return omp_get_max_threads(); }
