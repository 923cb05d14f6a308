// Lanczos ground state of H~ (App. Lanczos, Eqs. next_vector / an_bn,
// Eq. change_basis).
//
// The recurrence is kept in the paper's unnormalised form: u_0 = phi_0 and
// u_{k+1} = H v_k - a_k v_k - b_k v_{k-1} with v_k = u_k / ||u_k||, so
// b_k = ||u_k|| (k >= 1) and the tridiagonal H_eff has a_k on the diagonal
// and b_{k+1} next to it.  Normalisation is never a separate pass: the
// product kernel reads 1/||u_k|| from device memory and scales on the fly.
// Per step, two kernels:
//   apply (CSR stream or on-the-fly) : y = H v_k and a_k = <v_k|y>
//   k_lanczos_update                 : u_{k+1} = y - a_k v_k - b_k v_{k-1},
//                                      ||u_{k+1}||^2
// both with deterministic last-workgroup grid reductions, so the scalars
// never leave the GPU between convergence checks.  With store_vectors the
// u_k live in one [iters + 1][n] array in HBM and |Omega> = sum_k s_k v_k is
// one pass over it; otherwise the recurrence runs a second time and
// accumulates |Omega> (Eq. change_basis) without storage.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "mcd_hash.h"
#include "mcd_internal.h"
#include "mcd_reduce.h"
#include "mcd_tridiag.h"

namespace mcd {

static constexpr int BS = 256;

static inline unsigned nblk(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + BS - 1) / BS, 2048));
}

// phi0[r] = 2u - 1, u = top 53 bits of splitmix64's first output from state
// (seed XOR key_r).
__global__ void k_start_vector(int64_t n, const uint64_t *__restrict__ keys, uint64_t seed,
                               double *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    out[r] = start_value(keys[r], seed);
}

__global__ __launch_bounds__(BS) void k_dot(int64_t n, const double *__restrict__ a,
                                            const double *__restrict__ b,
                                            double *__restrict__ partials) {
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n; r += (int64_t)gridDim.x * BS)
        acc += a[r] * b[r];
    store_partial<BS>(block_sum<BS>(acc), partials);
}

__global__ __launch_bounds__(BS) void k_scale_dot(int64_t n, double *__restrict__ y,
                                                  const double *__restrict__ x,
                                                  const double *__restrict__ sx_dev, int sx_mode,
                                                  double *__restrict__ partials) {
    const double sx = scale_from(sx_dev, sx_mode);
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        const double v = y[r] * sx;
        y[r] = v;
        acc += x[r] * sx * v;
    }
    if (partials != nullptr) store_partial<BS>(block_sum<BS>(acc), partials);
}

// u_next = y - (a_k / ||u_k||) u_k - (||u_k|| / ||u_{k-1}||) u_{k-1};
// nrm2[k+1] = ||u_next||^2.  alpha, nrm2: device arrays of the recurrence.
__global__ __launch_bounds__(BS) void k_lanczos_update(
    int64_t n, int k, const double *__restrict__ y, const double *__restrict__ uk,
    const double *__restrict__ ukm1, double *__restrict__ unext, const double *__restrict__ alpha,
    const double *__restrict__ nrm2, double *__restrict__ partials) {
    const double ik = scale_from(&nrm2[k], 1);
    const double c1 = alpha[k] * ik;
    const double c2 = (k > 0) ? sqrt(nrm2[k]) * scale_from(&nrm2[k - 1], 1) : 0.0;
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        double w = y[r] - c1 * uk[r];
        if (k > 0) w -= c2 * ukm1[r];
        unext[r] = w;
        acc += w * w;
    }
    store_partial<BS>(block_sum<BS>(acc), partials);
}

// psi[r] = sum_k c_k U[k][r] (c_k = s_k / ||u_k||), one pass over the store.
__global__ __launch_bounds__(BS) void k_combine(int64_t n, int K, const double *__restrict__ U,
                                                const double *__restrict__ c,
                                                double *__restrict__ psi) {
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        double acc = 0.0;
        for (int k = 0; k < K; k++) acc += c[k] * U[(int64_t)k * n + r];
        psi[r] = acc;
    }
}

__global__ __launch_bounds__(BS) void k_axpy_coef(int64_t n, const double *__restrict__ c, int k,
                                                  const double *__restrict__ u,
                                                  double *__restrict__ psi, int first) {
    const double ck = c[k];
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS)
        psi[r] = first ? ck * u[r] : psi[r] + ck * u[r];
}

__global__ __launch_bounds__(BS) void k_scale(int64_t n, double *__restrict__ v,
                                              const double *__restrict__ nrm2) {
    const double s = scale_from(nrm2, 1);
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS)
        v[r] *= s;
}

int dev_dot(const mcd_op *op, const double *a, const double *b, int64_t n, double *out_dev,
            hipStream_t s) {
    hipLaunchKernelGGL(k_dot, dim3(nblk(n)), dim3(BS), 0, s, n, a, b, op->d_partials);
    hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nblk(n),
                       op->d_partials, out_dev);
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}

int scale_dot(const mcd_op *op, double *y, const double *x, const double *sx_dev, int sx_mode,
              double *dot_out, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_dot, dim3(nblk(op->n)), dim3(BS), 0, s, op->n, y, x, sx_dev,
                       sx_mode, dot_out ? op->d_partials : nullptr);
    if (dot_out)
        hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nblk(op->n),
                           op->d_partials, dot_out);
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}

// One Lanczos step k: reads u_k (and u_{k-1}), writes y and u_{k+1}.
static int lanczos_step(const mcd_op *op, int k, const double *uk, const double *ukm1,
                        double *unext, double *y, double *d_alpha, double *d_nrm2,
                        hipStream_t s) {
    MCD_TRY(apply_f64_fused(op, uk, y, &d_nrm2[k], 1, &d_alpha[k], s));
    hipLaunchKernelGGL(k_lanczos_update, dim3(nblk(op->n)), dim3(BS), 0, s, op->n, k, y, uk,
                       ukm1, unext, d_alpha, d_nrm2, op->d_partials);
    hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nblk(op->n),
                       op->d_partials, &d_nrm2[k + 1]);
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}

static double wall_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace mcd

using namespace mcd;

extern "C" int mcd_lanczos_ground(const mcd_op *op, const mcd_lanczos_cfg *cfg,
                                  const double *phi0_dev, double *e0, double *psi0_dev,
                                  double *alpha_out, double *beta_out, mcd_solve_info *info,
                                  void *stream) {
    MCD_REQUIRE(op && cfg && e0, MCD_E_INVALID, "op, cfg or e0 is NULL");
    MCD_REQUIRE(cfg->max_iter >= 1 && cfg->max_iter <= 100000, MCD_E_INVALID,
                "max_iter = %d outside 1..100000", cfg->max_iter);
    MCD_REQUIRE(op->n >= 1, MCD_E_INVALID, "empty basis");
    hipStream_t s = (hipStream_t)stream;
    const double t_start = wall_ms();
    const int64_t n = op->n;
    const int maxit = (int)std::min<int64_t>(cfg->max_iter, n);
    const int every = std::max(1, cfg->check_every);

    // Vector storage: the whole Krylov store if it fits half the free HBM
    // (the operator's workspace is reused between calls).
    size_t fr = 0, tot = 0;
    MCD_HIP(hipMemGetInfo(&fr, &tot));
    const size_t have = op->ws_bytes;
    const size_t sc_bytes = (3 * (size_t)maxit + 4) * sizeof(double);
    const size_t need_store = ((size_t)(maxit + 2) * n) * sizeof(double) + sc_bytes;
    bool store = cfg->store_vectors != 0 && (double)need_store < 0.5 * ((double)fr + have);
    const int64_t nvecs = store ? (maxit + 1) : 3;
    const size_t need = ((size_t)(nvecs + 1) * n) * sizeof(double) + sc_bytes;
    void *wsp = nullptr;
    MCD_TRY(op_workspace(op, need, &wsp));
    double *U = (double *)wsp;
    double *y = U + nvecs * n;
    double *d_sc = y + n;
    auto cleanup = [&]() {};
#define CK(expr)                                                                   \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));              \
            cleanup();                                                             \
            return MCD_E_HIP;                                                      \
        }                                                                          \
    } while (0)
#define TRY(expr)              \
    do {                       \
        int rc_ = (expr);      \
        if (rc_ < 0) {         \
            cleanup();         \
            return rc_;        \
        }                      \
    } while (0)
    double *d_alpha = d_sc, *d_nrm2 = d_sc + maxit, *d_coef = d_sc + 2 * maxit + 1;
    double *d_pn = d_sc + 3 * maxit + 2;
    auto vec = [&](int k) -> double * { return U + (store ? (int64_t)k : (int64_t)(k % 3)) * n; };

    if (phi0_dev)
        CK(hipMemcpyAsync(vec(0), phi0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    else
        hipLaunchKernelGGL(k_start_vector, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, s, n,
                           op->d_keys, cfg->seed, vec(0));
    TRY(dev_dot(op, vec(0), vec(0), n, &d_nrm2[0], s));

    hipEvent_t ev0, ev1;
    CK(hipEventCreate(&ev0));
    CK(hipEventCreate(&ev1));
    CK(hipEventRecord(ev0, s));
    std::vector<double> ha(maxit), hn2(maxit + 1);
    double lam = 0.0, resid = INFINITY;
    std::vector<double> svec;
    int K = 0;
    bool conv = false;
    for (int k = 0; k < maxit; k++) {
        TRY(lanczos_step(op, k, vec(k), k > 0 ? vec(k - 1) : vec(k), vec(k + 1), y, d_alpha,
                         d_nrm2, s));
        const bool check = ((k + 1) % every == 0) || (k + 1 == maxit);
        if (!check) continue;
        CK(hipMemcpyAsync(ha.data(), d_alpha, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(hn2.data(), d_nrm2, (k + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        // H_eff of size k+1: diagonal a_0..a_k, off-diagonal b_1..b_k.
        int m = k + 1;
        std::vector<double> b(m);
        for (int i = 1; i < m; i++) b[i] = sqrt(hn2[i]);
        // Breakdown: an earlier b_i ~ 0 ends the Krylov space there.
        double scale = 0.0;
        for (int i = 0; i < m; i++) scale = std::max(scale, fabs(ha[i]));
        int mb = m;
        for (int i = 1; i < m; i++)
            if (b[i] <= 1e-14 * std::max(1.0, scale)) {
                mb = i;
                break;
            }
        lam = tri_lowest(ha.data(), b.data(), mb);
        svec = tri_vector(ha.data(), b.data(), mb, lam);
        const double bnext = (mb < m) ? 0.0 : sqrt(hn2[m]);
        resid = bnext * fabs(svec[mb - 1]);
        K = mb;
        if (mb < m || bnext <= 1e-14 * std::max(1.0, scale)) {
            conv = true;
            break;
        }
        if (m >= cfg->min_iter && resid <= cfg->tol * std::max(1.0, fabs(lam))) {
            conv = true;
            break;
        }
    }
    CK(hipEventRecord(ev1, s));
    CK(hipEventSynchronize(ev1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);

    *e0 = lam;
    if (alpha_out) memcpy(alpha_out, ha.data(), K * sizeof(double));
    if (beta_out)
        for (int i = 0; i < K; i++) beta_out[i] = sqrt(hn2[i + 1]);

    if (psi0_dev) {
        std::vector<double> c(K);
        for (int k = 0; k < K; k++) c[k] = svec[k] / sqrt(hn2[k]);
        CK(hipMemcpyAsync(d_coef, c.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
        if (store) {
            hipLaunchKernelGGL(k_combine, dim3(nblk(n)), dim3(BS), 0, s, n, K, U, d_coef,
                               psi0_dev);
        } else {
            // Second pass of the recurrence (Eq. change_basis without storage).
            if (phi0_dev)
                CK(hipMemcpyAsync(vec(0), phi0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            else
                hipLaunchKernelGGL(k_start_vector, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS),
                                   0, s, n, op->d_keys, cfg->seed, vec(0));
            for (int k = 0; k < K; k++) {
                hipLaunchKernelGGL(k_axpy_coef, dim3(nblk(n)), dim3(BS), 0, s, n, d_coef, k,
                                   vec(k), psi0_dev, k == 0 ? 1 : 0);
                if (k + 1 < K)
                    TRY(lanczos_step(op, k, vec(k), k > 0 ? vec(k - 1) : vec(k), vec(k + 1), y,
                                     d_alpha, d_nrm2, s));
            }
        }
        TRY(dev_dot(op, psi0_dev, psi0_dev, n, d_pn, s));
        hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(BS), 0, s, n, psi0_dev, d_pn);
        CK(hipGetLastError());
    }
    CK(hipStreamSynchronize(s));
    cleanup();
#undef CK
#undef TRY
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = K;
        info->converged = conv ? 1 : 0;
        info->e0 = lam;
        info->residual = resid;
        info->solve_ms = wall_ms() - t_start;
        info->apply_ms = ms;
        info->n_apply = K;
        info->krylov_dim = K;
    }
    return conv ? MCD_OK : MCD_NOCONV;
}
