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
#include <cmath>
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
// (seed XOR key_r) (rounded to T).
template <typename T>
__global__ void k_start_vector(int64_t n, const uint64_t *__restrict__ keys, uint64_t seed,
                               T *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    out[r] = (T)start_value(keys[r], seed);
}

template <typename T>
__global__ void k_convert_vec(int64_t n, const double *__restrict__ in, T *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = (T)in[r];
}

template <typename T>
__global__ __launch_bounds__(BS) void k_dot(int64_t n, const T *__restrict__ a,
                                            const T *__restrict__ b,
                                            double *__restrict__ partials) {
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n; r += (int64_t)gridDim.x * BS)
        acc += (double)a[r] * (double)b[r];
    store_partial<BS>(block_sum<BS>(acc), partials);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_scale_dot(int64_t n, T *__restrict__ y,
                                                  const T *__restrict__ x,
                                                  const double *__restrict__ sx_dev, int sx_mode,
                                                  double *__restrict__ partials) {
    const double sx = scale_from(sx_dev, sx_mode);
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        const T v = y[r] * (T)sx;
        y[r] = v;
        acc += (double)x[r] * sx * (double)v;
    }
    if (partials != nullptr) store_partial<BS>(block_sum<BS>(acc), partials);
}

// u_next = y - (a_k / ||u_k||) u_k - (||u_k|| / ||u_{k-1}||) u_{k-1};
// nrm2[k+1] = ||u_next||^2.  alpha, nrm2: device arrays of the recurrence
// (float64); the vectors are T (the update is formed in float64 and rounded).
template <typename T>
__global__ __launch_bounds__(BS) void k_lanczos_update(
    int64_t n, int k, const T *__restrict__ y, const T *__restrict__ uk,
    const T *__restrict__ ukm1, T *__restrict__ unext, const double *__restrict__ alpha,
    const double *__restrict__ nrm2, double *__restrict__ partials) {
    const double ik = scale_from(&nrm2[k], 1);
    const double c1 = alpha[k] * ik;
    const double c2 = (k > 0) ? sqrt(nrm2[k]) * scale_from(&nrm2[k - 1], 1) : 0.0;
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        double w = (double)y[r] - c1 * (double)uk[r];
        if (k > 0) w -= c2 * (double)ukm1[r];
        const T wt = (T)w;
        unext[r] = wt;
        acc += (double)wt * (double)wt;
    }
    store_partial<BS>(block_sum<BS>(acc), partials);
}

// psi[r] = sum_k c_k U[k][r] (c_k = s_k / ||u_k||), one pass over the store
// (float64 accumulation and output).
template <typename T>
__global__ __launch_bounds__(BS) void k_combine(int64_t n, int K, const T *__restrict__ U,
                                                const double *__restrict__ c,
                                                double *__restrict__ psi) {
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        double acc = 0.0;
        for (int k = 0; k < K; k++) acc += c[k] * (double)U[(int64_t)k * n + r];
        psi[r] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_axpy_coef(int64_t n, const double *__restrict__ c, int k,
                                                  const T *__restrict__ u,
                                                  double *__restrict__ psi, int first) {
    const double ck = c[k];
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS)
        psi[r] = first ? ck * (double)u[r] : psi[r] + ck * (double)u[r];
}

__global__ __launch_bounds__(BS) void k_scale(int64_t n, double *__restrict__ v,
                                              const double *__restrict__ nrm2) {
    const double s = scale_from(nrm2, 1);
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS)
        v[r] *= s;
}

// Partials of ||y - e psi||^2 with e = *e_dev (the residual of a Ritz pair).
__global__ __launch_bounds__(BS) void k_resid2(int64_t n, const double *__restrict__ y,
                                               const double *__restrict__ psi,
                                               const double *__restrict__ e_dev,
                                               double *__restrict__ partials) {
    const double e = *e_dev;
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS) {
        const double d = y[r] - e * psi[r];
        acc += d * d;
    }
    store_partial<BS>(block_sum<BS>(acc), partials);
}

template <typename T>
static int dot_t(const mcd_op *op, const T *a, const T *b, int64_t n, double *out_dev,
                 hipStream_t s) {
    hipLaunchKernelGGL((k_dot<T>), dim3(nblk(n)), dim3(BS), 0, s, n, a, b, op->d_partials);
    hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nblk(n),
                       op->d_partials, out_dev);
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}

int dev_dot(const mcd_op *op, const double *a, const double *b, int64_t n, double *out_dev,
            hipStream_t s) {
    return dot_t<double>(op, a, b, n, out_dev, s);
}

template <typename T>
int scale_dot(const mcd_op *op, T *y, const T *x, const double *sx_dev, int sx_mode,
              double *dot_out, hipStream_t s) {
    hipLaunchKernelGGL((k_scale_dot<T>), dim3(nblk(op->n)), dim3(BS), 0, s, op->n, y, x, sx_dev,
                       sx_mode, dot_out ? op->d_partials : nullptr);
    if (dot_out)
        hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nblk(op->n),
                           op->d_partials, dot_out);
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}
template int scale_dot<double>(const mcd_op *, double *, const double *, const double *, int,
                               double *, hipStream_t);
template int scale_dot<float>(const mcd_op *, float *, const float *, const double *, int,
                              double *, hipStream_t);

// One Lanczos step k: reads u_k (and u_{k-1}), writes y and u_{k+1}.
template <typename T>
static int lanczos_step(const mcd_op *op, int k, const T *uk, const T *ukm1, T *unext, T *y,
                        double *d_alpha, double *d_nrm2, hipStream_t s) {
    MCD_TRY(apply_fused<T>(op, uk, y, &d_nrm2[k], 1, &d_alpha[k], s));
    hipLaunchKernelGGL((k_lanczos_update<T>), dim3(nblk(op->n)), dim3(BS), 0, s, op->n, k, y, uk,
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

// Workspace layout of one solve: [vectors: nvecs][y][refinement y64][scalars]
struct LzLayout {
    int maxit;
    int64_t nvecs;
    size_t vec_bytes, y_bytes, y64_bytes, sc_bytes;
    size_t total() const { return vec_bytes + y_bytes + y64_bytes + sc_bytes; }
};
static LzLayout lz_layout(const mcd_op *op, const mcd_lanczos_cfg *cfg) {
    LzLayout L;
    const int64_t n = op->n;
    L.maxit = (int)std::min<int64_t>(cfg->max_iter, n);
    const bool store = cfg->store_vectors != 0;
    const size_t es = cfg->precision == MCD_F32 ? sizeof(float) : sizeof(double);
    L.nvecs = store ? (L.maxit + 1) : 3;
    L.vec_bytes = WsAlloc::round((size_t)L.nvecs * n * es);
    L.y_bytes = WsAlloc::round((size_t)n * es);
    L.y64_bytes = cfg->precision == MCD_F32 ? WsAlloc::round((size_t)n * sizeof(double)) : 0;
    L.sc_bytes = WsAlloc::round((3 * (size_t)L.maxit + 8) * sizeof(double));
    return L;
}

template <typename T>
static int lanczos_run(const mcd_op *op, const mcd_lanczos_cfg *cfg, const double *phi0_dev,
                       double *e0, double *psi0_dev, double *alpha_out, double *beta_out,
                       mcd_solve_info *info, mcd_ws *ws, hipStream_t s) {
    const double t_start = wall_ms();
    const int64_t n = op->n;
    const LzLayout L = lz_layout(op, cfg);
    const int maxit = L.maxit;
    const int every = std::max(1, cfg->check_every);
    const bool store = cfg->store_vectors != 0;
    const bool refine = sizeof(T) == sizeof(float);
    const Alloc al{ws};
    char *wsp = nullptr;
    MCD_HIP(dmalloc((void **)&wsp, L.total(), al));
    if (poison_fp(wsp, L.total(), al, s) != hipSuccess) {
        (void)dfree(wsp, al);
        set_error("lanczos: workspace fill failed");
        return MCD_E_HIP;
    }
    T *U = (T *)wsp;
    T *y = (T *)(wsp + L.vec_bytes);
    double *y64 = (double *)(wsp + L.vec_bytes + L.y_bytes);
    double *d_sc = (double *)(wsp + L.vec_bytes + L.y_bytes + L.y64_bytes);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);   // queued work reads the pieces
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        (void)dfree(wsp, al);
    };
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
    double *d_pn = d_sc + 3 * maxit + 2, *d_e = d_pn + 1, *d_r2 = d_pn + 2;
    auto vec = [&](int k) -> T * { return U + (store ? (int64_t)k : (int64_t)(k % 3)) * n; };
    auto start = [&]() -> int {
        if (phi0_dev) {
            if (sizeof(T) == sizeof(double)) {
                MCD_HIP(hipMemcpyAsync(vec(0), phi0_dev, n * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
            } else {
                hipLaunchKernelGGL((k_convert_vec<T>), dim3((unsigned)((n + BS - 1) / BS)),
                                   dim3(BS), 0, s, n, phi0_dev, vec(0));
            }
        } else {
            hipLaunchKernelGGL((k_start_vector<T>), dim3((unsigned)((n + BS - 1) / BS)), dim3(BS),
                               0, s, n, op->d_keys, cfg->seed, vec(0));
        }
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    };
    TRY(start());
    TRY(dot_t<T>(op, vec(0), vec(0), n, &d_nrm2[0], s));

    CK(hipEventCreate(&ev0));
    CK(hipEventCreate(&ev1));
    CK(hipEventRecord(ev0, s));
    std::vector<double> ha(maxit), hn2(maxit + 1);
    double lam = 0.0, resid = INFINITY;
    std::vector<double> svec;
    int K = 0;
    bool conv = false;
    for (int k = 0; k < maxit; k++) {
        TRY(lanczos_step<T>(op, k, vec(k), k > 0 ? vec(k - 1) : vec(k), vec(k + 1), y, d_alpha,
                            d_nrm2, s));
        const bool check = ((k + 1) % every == 0) || (k + 1 == maxit);
        if (!check) continue;
        CK(hipMemcpyAsync(ha.data(), d_alpha, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(hn2.data(), d_nrm2, (k + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        int m = k + 1;
        for (int i = 0; i <= m && i < (int)hn2.size(); i++)
            if (!std::isfinite(hn2[i]) || (i < m && !std::isfinite(ha[i]))) {
                cleanup();
                set_error("Lanczos: non-finite coefficient at step %d (NaN or Inf in the start "
                          "vector or the operator)", i);
                return MCD_E_NUMERIC;
            }
        // H_eff of size k+1: diagonal a_0..a_k, off-diagonal b_1..b_k.
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

    if (alpha_out) memcpy(alpha_out, ha.data(), K * sizeof(double));
    if (beta_out)
        for (int i = 0; i < K; i++) beta_out[i] = sqrt(hn2[i + 1]);

    // the Ritz vector (float64): needed for psi0 and for the refinement
    double *psi = psi0_dev ? psi0_dev : (refine ? y64 : nullptr);
    double *yr = refine ? (psi0_dev ? y64 : nullptr) : nullptr;
    std::vector<double> c(K);   // lives until the synchronisation below
    if (psi) {
        for (int k = 0; k < K; k++) c[k] = svec[k] / sqrt(hn2[k]);
        CK(hipMemcpyAsync(d_coef, c.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
        if (store) {
            hipLaunchKernelGGL((k_combine<T>), dim3(nblk(n)), dim3(BS), 0, s, n, K, U, d_coef, psi);
        } else {
            // Second pass of the recurrence (Eq. change_basis without storage).
            TRY(start());
            for (int k = 0; k < K; k++) {
                hipLaunchKernelGGL((k_axpy_coef<T>), dim3(nblk(n)), dim3(BS), 0, s, n, d_coef, k,
                                   vec(k), psi, k == 0 ? 1 : 0);
                if (k + 1 < K)
                    TRY(lanczos_step<T>(op, k, vec(k), k > 0 ? vec(k - 1) : vec(k), vec(k + 1), y,
                                        d_alpha, d_nrm2, s));
            }
        }
        TRY(dev_dot(op, psi, psi, n, d_pn, s));
        hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(BS), 0, s, n, psi, d_pn);
        CK(hipGetLastError());
    }
    double e_ritz = lam;
    if (refine) {
        // E0 = <psi|H~|psi> of the normalised float64 Ritz vector from one
        // float64 product, and its true residual ||H~ psi - E0 psi||.
        if (yr == nullptr) {   // psi lives in y64: the product goes to the float32 store
            // (only reached without psi0_dev: reuse the first two float vectors
            // as one float64 vector of n entries)
            yr = (double *)U;
        }
        TRY(apply_fused<double>(op, psi, yr, nullptr, 0, d_e, s));
        hipLaunchKernelGGL(k_resid2, dim3(nblk(n)), dim3(BS), 0, s, n, yr, psi, d_e,
                           op->d_partials);
        hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nblk(n),
                           op->d_partials, d_r2);
        CK(hipGetLastError());
        double er[2] = {0.0, 0.0};
        CK(hipMemcpyAsync(er, d_e, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        lam = er[0];
        resid = sqrt(std::max(er[1], 0.0));
        if (!std::isfinite(lam)) {
            cleanup();
            set_error("Lanczos: non-finite Rayleigh quotient in the float64 refinement");
            return MCD_E_NUMERIC;
        }
    }
    CK(hipStreamSynchronize(s));
    cleanup();
#undef CK
#undef TRY
    *e0 = lam;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = K;
        info->converged = conv ? 1 : 0;
        info->e0 = lam;
        info->residual = resid;
        info->solve_ms = wall_ms() - t_start;
        info->apply_ms = ms;
        info->n_apply = K + (refine ? 1 : 0);
        info->krylov_dim = K;
    }
    (void)e_ritz;
    return conv ? MCD_OK : MCD_NOCONV;
}

}  // namespace mcd

using namespace mcd;

extern "C" int mcd_lanczos_workspace_size(const mcd_op *op, const mcd_lanczos_cfg *cfg,
                                          size_t *bytes) {
    MCD_REQUIRE(op && cfg && bytes, MCD_E_INVALID, "op, cfg or bytes is NULL");
    MCD_REQUIRE(cfg->max_iter >= 1 && cfg->max_iter <= 100000, MCD_E_INVALID,
                "max_iter = %d outside 1..100000", cfg->max_iter);
    MCD_REQUIRE(cfg->precision == MCD_F64 || cfg->precision == MCD_F32, MCD_E_INVALID,
                "precision must be MCD_F64 or MCD_F32");
    *bytes = lz_layout(op, cfg).total();
    return MCD_OK;
}

extern "C" int mcd_lanczos_ground(const mcd_op *op, const mcd_lanczos_cfg *cfg,
                                  const double *phi0_dev, double *e0, double *psi0_dev,
                                  double *alpha_out, double *beta_out, mcd_solve_info *info,
                                  mcd_ws *ws, void *stream) {
    MCD_REQUIRE(op && cfg && e0, MCD_E_INVALID, "op, cfg or e0 is NULL");
    MCD_REQUIRE(cfg->max_iter >= 1 && cfg->max_iter <= 100000, MCD_E_INVALID,
                "max_iter = %d outside 1..100000", cfg->max_iter);
    MCD_REQUIRE(op->n >= 1, MCD_E_INVALID, "empty basis");
    MCD_REQUIRE(cfg->precision == MCD_F64 || cfg->precision == MCD_F32, MCD_E_INVALID,
                "precision must be MCD_F64 or MCD_F32");
    if (cfg->precision == MCD_F32) {
        // the refinement's float64 product goes to the float32 vector store
        // when psi0 is not requested: it must hold n doubles
        MCD_REQUIRE(psi0_dev != nullptr || lz_layout(op, cfg).vec_bytes >= (size_t)op->n * 8,
                    MCD_E_INVALID, "float32 Lanczos without psi0 needs >= 2 stored vectors");
        return lanczos_run<float>(op, cfg, phi0_dev, e0, psi0_dev, alpha_out, beta_out, info, ws,
                                  (hipStream_t)stream);
    }
    return lanczos_run<double>(op, cfg, phi0_dev, e0, psi0_dev, alpha_out, beta_out, info, ws,
                               (hipStream_t)stream);
}
