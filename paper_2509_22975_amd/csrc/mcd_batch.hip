// Batched Lanczos ground states of many independent operators (bath
// instances of uneven basis size, App. Lanczos for each).
//
// All recurrences advance together: one step is five launches for the whole
// batch, whatever the number of instances --
//   k_bspmv    y_i = H_i v_k(i) for every instance (row blocks of all
//              instances in one grid, each block tagged with its instance),
//              with per-block partials of <v_k(i)|y_i>;
//   k_bfinal   per-instance sums of the partials -> a_k(i);
//   k_bupdate  u_{k+1}(i) = y_i - a_k v_k - b_k v_{k-1}, partials of ||.||^2;
//   k_bfinal   -> ||u_{k+1}(i)||^2;
//   k_bstep    advance the device-resident step counter.
// Kernel arguments never change between steps (the step index lives on the
// device), so `check_every` steps are captured once into a HIP graph and the
// graph is replayed; converged instances are switched off through a device
// flag and their blocks return at once.  Reductions are per-block partials
// summed in index order: deterministic.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "mcd_hash.h"
#include "mcd_internal.h"
#include "mcd_reduce.h"
#include "mcd_tridiag.h"

namespace mcd {

static constexpr int BBS = 256;
static constexpr int kUpdRows = 2048;   // rows per update workgroup

struct BDesc {
    const int64_t *rowptr;
    const uint32_t *colw;
    const double *diag;
    const DevModel *m;
    const uint64_t *keys;
    int64_t n;
    int64_t blk0;      // first SpMV block of the instance
    int64_t ublk0;     // first update block
    int64_t ubase;     // offset of the instance's Krylov store
    int64_t row0;      // offset of the instance's rows in y
};

struct BState {
    const BDesc *d;
    int K;             // instances
    int R;             // rows per SpMV block
    int stride;        // scalars per instance (max_iter + 1)
    double *U;         // Krylov stores
    double *Y;         // products
    double *alpha;     // [K][stride]
    double *nrm2;      // [K][stride]
    double *partials;
    const int *active;
    const int *kdev;   // current step
};

__device__ __forceinline__ int find_inst(const BDesc *__restrict__ d, int K, int64_t b,
                                         bool upd) {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t start = upd ? d[mid].ublk0 : d[mid].blk0;
        if (start <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(BBS) void k_bspmv(BState st) {
    __shared__ double prod[kStreamNnzMax];
    __shared__ double vtab[kMaxClasses];
    constexpr int DEPTH = kStreamNnzMax / BBS;
    const int tid = threadIdx.x;
    const int inst = find_inst(st.d, st.K, blockIdx.x, false);
    const BDesc &D = st.d[inst];
    if (!st.active[inst]) {
        if (tid == 0) st.partials[blockIdx.x] = 0.0;
        return;
    }
    const int k = *st.kdev;
    const double *__restrict__ x = st.U + D.ubase + (int64_t)k * D.n;
    double *__restrict__ y = st.Y + D.row0;
    const double sx = scale_from(&st.nrm2[inst * st.stride + k], 1);
    const int64_t r0 = (blockIdx.x - D.blk0) * (int64_t)st.R;
    const int64_t r1 = min(r0 + (int64_t)st.R, D.n);
    // Unconditional loads on clamped addresses (as in the one-operator stream
    // kernel): no branches around loads, waits by count.
    const bool own = tid < st.R && r0 + tid < r1;
    const int64_t r = min(r0 + (int64_t)tid, r1 - 1);
    const int64_t rs = D.rowptr[r], re = D.rowptr[r + 1];
    const double dr = D.diag[r], xr = x[r];
    if (tid < kMaxClasses) vtab[tid] = D.m->vtab[tid];
    const uint32_t cmask = D.m->col_mask, cbits = D.m->col_bits;
    const int64_t e0 = D.rowptr[r0];
    const int cnt = (int)(D.rowptr[r1] - e0);
    const uint32_t *__restrict__ cw = D.colw + e0;
    uint32_t w[DEPTH];
    double xv[DEPTH];
    if (cnt > 0) {   // uniform over the workgroup
#pragma unroll
        for (int j = 0; j < DEPTH; j++) w[j] = cw[min(tid + j * BBS, cnt - 1)];
#pragma unroll
        for (int j = 0; j < DEPTH; j++) xv[j] = x[w[j] & cmask];
    }
    __syncthreads();
    if (cnt > 0) {
#pragma unroll
        for (int j = 0; j < DEPTH; j++) {
            const int e = tid + j * BBS;
            if (e < cnt) {
                const double v = vtab[(w[j] & 0x7fffffffu) >> cbits];
                prod[e] = (w[j] >> 31) ? -(v * xv[j]) : v * xv[j];
            }
        }
    }
    __syncthreads();
    double dot = 0.0;
    if (own) {
        double acc = dr * xr;
        for (int q = (int)(rs - e0); q < (int)(re - e0); q++) acc += prod[q];
        acc *= sx;
        y[r] = acc;
        dot = xr * sx * acc;
    }
    store_partial<BBS>(block_sum<BBS>(dot), st.partials);
}

// out[i * stride + k + koff] = sum of instance i's block partials (index order).
__global__ __launch_bounds__(BBS) void k_bfinal(BState st, int upd, double *out, int koff) {
    const int inst = blockIdx.x;
    if (!st.active[inst]) return;
    const BDesc &D = st.d[inst];
    const int64_t b0 = upd ? D.ublk0 : D.blk0;
    const int64_t nb = upd ? (D.n + kUpdRows - 1) / kUpdRows : (D.n + st.R - 1) / st.R;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += BBS) s += st.partials[b0 + i];
    s = block_sum<BBS>(s);
    if (threadIdx.x == 0) out[inst * st.stride + *st.kdev + koff] = s;
}

__global__ __launch_bounds__(BBS) void k_bupdate(BState st) {
    const int inst = find_inst(st.d, st.K, blockIdx.x, true);
    const BDesc &D = st.d[inst];
    if (!st.active[inst]) {
        if (threadIdx.x == 0) st.partials[blockIdx.x] = 0.0;
        return;
    }
    const int k = *st.kdev;
    const double *__restrict__ y = st.Y + D.row0;
    const double *__restrict__ uk = st.U + D.ubase + (int64_t)k * D.n;
    const double *__restrict__ ukm1 = st.U + D.ubase + (int64_t)(k > 0 ? k - 1 : 0) * D.n;
    double *__restrict__ un = st.U + D.ubase + (int64_t)(k + 1) * D.n;
    const double *nr = st.nrm2 + inst * st.stride;
    const double c1 = st.alpha[inst * st.stride + k] * scale_from(&nr[k], 1);
    const double c2 = (k > 0) ? sqrt(nr[k]) * scale_from(&nr[k - 1], 1) : 0.0;
    const int64_t r0 = (blockIdx.x - D.ublk0) * (int64_t)kUpdRows;
    const int64_t r1 = min(r0 + (int64_t)kUpdRows, D.n);
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BBS) {
        double w = y[r] - c1 * uk[r];
        if (k > 0) w -= c2 * ukm1[r];
        un[r] = w;
        acc += w * w;
    }
    store_partial<BBS>(block_sum<BBS>(acc), st.partials);
}

__global__ void k_bstep(int *kdev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *kdev += 1;
}

__global__ void k_bstart(int64_t n, const uint64_t *__restrict__ keys, uint64_t seed,
                         double *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = start_value(keys[r], seed);
}

__global__ __launch_bounds__(BBS) void k_bnorm0(BState st) {
    // partial of ||u_0||^2 per update block (same tiling as k_bupdate)
    const int inst = find_inst(st.d, st.K, blockIdx.x, true);
    const BDesc &D = st.d[inst];
    const double *__restrict__ u = st.U + D.ubase;
    const int64_t r0 = (blockIdx.x - D.ublk0) * (int64_t)kUpdRows;
    const int64_t r1 = min(r0 + (int64_t)kUpdRows, D.n);
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BBS) acc += u[r] * u[r];
    store_partial<BBS>(block_sum<BBS>(acc), st.partials);
}

__global__ __launch_bounds__(BBS) void k_bcombine(int64_t n, int K, const double *__restrict__ U,
                                                  const double *__restrict__ c,
                                                  double *__restrict__ psi) {
    for (int64_t r = (int64_t)blockIdx.x * BBS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BBS) {
        double acc = 0.0;
        for (int k = 0; k < K; k++) acc += c[k] * U[(int64_t)k * n + r];
        psi[r] = acc;
    }
}

// Normalising psi: workgroup partial sums of squares (grid-stride, fixed
// order), k_finalize_sum into a device scalar, then v *= 1 / sqrt(sum).
__global__ __launch_bounds__(BBS) void k_bsumsq(int64_t n, const double *__restrict__ v,
                                                double *__restrict__ partials) {
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BBS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BBS)
        acc += v[r] * v[r];
    store_partial<BBS>(block_sum<BBS>(acc), partials);
}

__global__ __launch_bounds__(BBS) void k_bscale(int64_t n, double *__restrict__ v,
                                                const double *__restrict__ nrm2) {
    const double s = scale_from(nrm2, 1);
    for (int64_t r = (int64_t)blockIdx.x * BBS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BBS)
        v[r] *= s;
}

static double bwall_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace mcd

using namespace mcd;

extern "C" int mcd_batch_lanczos_ground(mcd_op *const *ops, int32_t n_ops,
                                        const mcd_lanczos_cfg *cfg, double *e0_out,
                                        double *const *psi0_dev, int32_t *iters_out,
                                        mcd_solve_info *info, mcd_ws *ws, void *stream) {
    MCD_REQUIRE(ops && cfg && e0_out && n_ops >= 1 && n_ops <= 4096, MCD_E_INVALID,
                "ops, cfg, e0_out required; 1 <= n_ops <= 4096");
    MCD_REQUIRE(cfg->precision == MCD_F64, MCD_E_INVALID, "batched Lanczos is float64 only");
    const double t_start = bwall_ms();
    const int K = n_ops;
    int R = 256;
    int64_t Ntot = 0, nmax = 0;
    for (int i = 0; i < K; i++) {
        MCD_REQUIRE(ops[i] && ops[i]->storage == MCD_STORAGE_CSR && ops[i]->n >= 1, MCD_E_INVALID,
                    "operator %d must be a non-empty CSR operator", i);
        R = std::min(R, (int)ops[i]->rows_per_block);
        Ntot += ops[i]->n;
        nmax = std::max(nmax, ops[i]->n);
    }
    const int maxit = (int)std::min<int64_t>(cfg->max_iter, nmax);
    MCD_REQUIRE(maxit >= 1, MCD_E_INVALID, "max_iter must be >= 1");
    const int stride = maxit + 1;
    const int every = std::max(1, cfg->check_every);
    // Layout and block tables.
    std::vector<BDesc> hd(K);
    int64_t nb = 0, ub = 0, row0 = 0;
    for (int i = 0; i < K; i++) {
        const mcd_op *op = ops[i];
        hd[i] = BDesc{op->d_rowptr, op->d_colw, op->d_diag, op->d_model, op->d_keys, op->n,
                      nb, ub, (int64_t)stride * row0, row0};
        nb += (op->n + R - 1) / R;
        ub += (op->n + kUpdRows - 1) / kUpdRows;
        row0 += op->n;
    }
    const size_t store_bytes = (size_t)stride * Ntot * sizeof(double);
    const Alloc al{ws};
    hipStream_t s = (hipStream_t)stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    BDesc *dd = nullptr;
    double *U = nullptr, *Y = nullptr, *sc = nullptr, *part = nullptr, *coef = nullptr;
    int *iv = nullptr;
    auto cleanup = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamSynchronize(s);   // queued work reads the pieces
        for (void *p : {(void *)dd, (void *)U, (void *)Y, (void *)sc, (void *)part, (void *)coef,
                        (void *)iv})
            if (p) (void)dfree(p, al);
    };
#define CK(expr)                                                              \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess) {                                               \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
            cleanup();                                                        \
            return hip_status(e_);                                            \
        }                                                                     \
    } while (0)
    CK(dmalloc((void **)&dd, K * sizeof(BDesc), al));
    CK(hipMemcpyAsync(dd, hd.data(), K * sizeof(BDesc), hipMemcpyHostToDevice, s));
    CK(dmalloc((void **)&U, store_bytes, al));
    CK(dmalloc((void **)&Y, Ntot * sizeof(double), al));
    CK(dmalloc((void **)&sc, (size_t)2 * K * stride * sizeof(double), al));
    CK(poison_fp(U, store_bytes, al, s));
    CK(poison_fp(Y, Ntot * sizeof(double), al, s));
    CK(poison_fp(sc, (size_t)2 * K * stride * sizeof(double), al, s));
    CK(hipMemsetAsync(sc, 0, (size_t)2 * K * stride * sizeof(double), s));
    CK(dmalloc((void **)&part, std::max(nb, ub) * sizeof(double), al));
    CK(poison_fp(part, std::max(nb, ub) * sizeof(double), al, s));
    // psi coefficients of every instance, then the norm partials (at most
    // 2048 workgroups) and one squared norm per instance
    constexpr int kNormPart = 2048;
    CK(dmalloc((void **)&coef, ((size_t)K * stride + kNormPart + K) * sizeof(double), al));
    CK(poison_fp(coef, ((size_t)K * stride + kNormPart + K) * sizeof(double), al, s));
    CK(dmalloc((void **)&iv, (K + 1) * sizeof(int), al));
    std::vector<int> hact(K + 1, 1);
    hact[K] = 0;   // step counter
    CK(hipMemcpyAsync(iv, hact.data(), (K + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    BState st{dd, K, R, stride, U, Y, sc, sc + (size_t)K * stride, part, iv, iv + K};
    // start vectors and ||u_0||^2
    for (int i = 0; i < K; i++)
        hipLaunchKernelGGL(k_bstart, dim3((unsigned)((hd[i].n + 255) / 256)), dim3(256), 0, s,
                           hd[i].n, hd[i].keys, cfg->seed, U + hd[i].ubase);
    hipLaunchKernelGGL(k_bnorm0, dim3((unsigned)ub), dim3(BBS), 0, s, st);
    hipLaunchKernelGGL(k_bfinal, dim3(K), dim3(BBS), 0, s, st, 1, st.nrm2, 0);
    CK(hipGetLastError());

    auto enqueue_step = [&]() {
        hipLaunchKernelGGL(k_bspmv, dim3((unsigned)nb), dim3(BBS), 0, s, st);
        hipLaunchKernelGGL(k_bfinal, dim3(K), dim3(BBS), 0, s, st, 0, st.alpha, 0);
        hipLaunchKernelGGL(k_bupdate, dim3((unsigned)ub), dim3(BBS), 0, s, st);
        hipLaunchKernelGGL(k_bfinal, dim3(K), dim3(BBS), 0, s, st, 1, st.nrm2, 1);
        hipLaunchKernelGGL(k_bstep, dim3(1), dim3(64), 0, s, iv + K);
    };
    // One graph of `every` steps, captured on the caller's stream and
    // replayed; a stream that cannot be captured (the legacy NULL stream)
    // gets the same launches one by one.
    const int chunk = std::min(every, maxit);
    if (s != nullptr) {
        CK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int q = 0; q < chunk; q++) enqueue_step();
        CK(hipStreamEndCapture(s, &graph));
        CK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }

    hipEvent_t ev0, ev1;
    CK(hipEventCreate(&ev0));
    CK(hipEventCreate(&ev1));
    CK(hipEventRecord(ev0, s));
    std::vector<double> ha((size_t)K * stride), hn((size_t)K * stride);
    std::vector<int> Kdone(K, 0), conv(K, 0);
    std::vector<double> lam(K, 0.0), resid(K, INFINITY);
    std::vector<std::vector<double>> svec(K);
    int steps = 0;
    int n_active = K;
    while (steps < maxit && n_active > 0) {
        if (steps + chunk <= maxit) {
            if (gexec) {
                CK(hipGraphLaunch(gexec, s));
            } else {
                for (int q = 0; q < chunk; q++) enqueue_step();
            }
            steps += chunk;
        } else {
            enqueue_step();
            steps += 1;
        }
        CK(hipMemcpyAsync(ha.data(), st.alpha, ha.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(hn.data(), st.nrm2, hn.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        bool changed = false;
        for (int i = 0; i < K; i++) {
            if (!hact[i]) continue;
            const int m = std::min<int64_t>(steps, hd[i].n);
            const double *a = &ha[(size_t)i * stride];
            const double *n2 = &hn[(size_t)i * stride];
            std::vector<double> b(m);
            double scale = 0.0;
            for (int q = 0; q < m; q++) scale = std::max(scale, fabs(a[q]));
            int mb = m;
            for (int q = 1; q < m; q++) {
                b[q] = sqrt(n2[q]);
                if (b[q] <= 1e-14 * std::max(1.0, scale)) {
                    mb = q;
                    break;
                }
            }
            lam[i] = tri_lowest(a, b.data(), mb);
            svec[i] = tri_vector(a, b.data(), mb, lam[i]);
            const double bnext = (mb < m) ? 0.0 : sqrt(n2[m]);
            resid[i] = bnext * fabs(svec[i][mb - 1]);
            Kdone[i] = mb;
            const bool done = mb < m || bnext <= 1e-14 * std::max(1.0, scale) ||
                              (m >= cfg->min_iter && resid[i] <= cfg->tol * std::max(1.0, fabs(lam[i]))) ||
                              m >= hd[i].n;
            if (done) {
                conv[i] = (resid[i] <= cfg->tol * std::max(1.0, fabs(lam[i]))) || mb < m ||
                          bnext <= 1e-14 * std::max(1.0, scale) || m >= hd[i].n;
                hact[i] = 0;
                n_active--;
                changed = true;
            }
        }
        if (changed) CK(hipMemcpyAsync(iv, hact.data(), K * sizeof(int), hipMemcpyHostToDevice, s));
    }
    CK(hipEventRecord(ev1, s));
    CK(hipEventSynchronize(ev1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    int all_conv = 1, max_it = 0;
    // psi_i = sum_q (s_q / ||u_q||) u_q, normalised: all coefficients in one
    // upload (hc lives until the synchronisation below), then per instance
    // the combination, its norm and the scaling, with no host round trip
    std::vector<double> hc((size_t)K * stride, 0.0);
    for (int i = 0; i < K; i++) {
        e0_out[i] = lam[i];
        if (iters_out) iters_out[i] = Kdone[i];
        all_conv &= conv[i];
        max_it = std::max(max_it, Kdone[i]);
        if (psi0_dev && psi0_dev[i])
            for (int q = 0; q < Kdone[i]; q++)
                hc[(size_t)i * stride + q] = svec[i][q] / sqrt(hn[(size_t)i * stride + q]);
    }
    if (psi0_dev) {
        double *npart = coef + (size_t)K * stride, *nrm2 = npart + kNormPart;
        CK(hipMemcpyAsync(coef, hc.data(), hc.size() * sizeof(double), hipMemcpyHostToDevice, s));
        for (int i = 0; i < K; i++) {
            if (!psi0_dev[i]) continue;
            const int64_t ni = hd[i].n;
            const unsigned g = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>((ni + BBS - 1) / BBS, kNormPart));
            hipLaunchKernelGGL(k_bcombine, dim3(g), dim3(BBS), 0, s, ni, Kdone[i],
                               U + hd[i].ubase, coef + (size_t)i * stride, psi0_dev[i]);
            hipLaunchKernelGGL(k_bsumsq, dim3(g), dim3(BBS), 0, s, ni, psi0_dev[i], npart);
            hipLaunchKernelGGL((k_finalize_sum<BBS>), dim3(1), dim3(BBS), 0, s, (int)g, npart,
                               nrm2 + i);
            hipLaunchKernelGGL(k_bscale, dim3(g), dim3(BBS), 0, s, ni, psi0_dev[i], nrm2 + i);
            CK(hipGetLastError());
        }
    }
    CK(hipStreamSynchronize(s));
    cleanup();
#undef CK
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = max_it;
        info->converged = all_conv;
        info->solve_ms = bwall_ms() - t_start;
        info->apply_ms = ms;
        info->n_apply = steps;
        info->krylov_dim = max_it;
    }
    return all_conv ? MCD_OK : MCD_NOCONV;
}
