// Green function of the truncated ground state by block (band) Lanczos on
// the excited subspaces (Sec. Subspace of the Green function, Sec. Further
// truncation, App. Band Lanczos, Eqs. green_qmatrix / q_matrix).
//
// Pipeline (all vector work on the GPU, p x p algebra on the host):
//  1. target-weight cut of |Omega>: radix sort of |c_n|^2 (descending,
//     stable so ties stay in key order), cumulative weight on the host,
//     kept rows re-sorted by key and renormalised;
//  2. F~+ / F~-: images c+_mu x / c_mu x of every kept state for the selected
//     (orbital, spin) pairs, radix sort + unique (Eq. excited_subspace);
//  3. start block c+_mu|Omega> (c_mu|Omega>) scattered into F~+- through the
//     operator's hash, Jordan-Wigner sign of the ordering "up orbitals, then
//     down orbitals";
//  4. block Lanczos with block width P (the selected p padded to a power of
//     two; zero columns deflate at once): W = H Q_j (block SpMM), A_j = Q_j^T W,
//     W -= Q_j A_j + Q_{j-1} B_j^T, optional full reorthogonalisation against
//     every stored block (one or two passes), W = Q_{j+1} B_{j+1} by a
//     rank-revealing QR applied twice that drops directions of norm <= dtol
//     (the band method's deflation): pivoted Cholesky of the Gram matrix in
//     one wavefront for the block products, a Gram eigen-decomposition on
//     the host in the per-column reference form -- either way the columns
//     span the block Krylov space K_r^L;
//  5. G(z) = R^T [(z - T)^-1]_{00} R by a block continued fraction over the
//     block tridiagonal T (complex128, host), z = i w + E0 for G+ and
//     G- = -R^T [(E0 - i w) - T]^-1 R; this is the resolvent that the Lehmann
//     sums of Eqs. green_qmatrix write through the eigenpairs of T.
#include <hipcub/hipcub.hpp>
#include <math.h>

#include <cmath>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <complex>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mcd_hash.h"
#include "mcd_internal.h"
#include "mcd_reduce.h"
#include "mcd_spmm.h"

namespace mcd {

using cplx = std::complex<double>;
static constexpr int BS = 256;

static inline unsigned gridn(int64_t n, int bs) {
    return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs);
}

__global__ void k_weights(int64_t n, const double *__restrict__ psi, double *__restrict__ w,
                          uint32_t *__restrict__ idx) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    w[r] = psi[r] * psi[r];
    idx[r] = (uint32_t)r;
}

__global__ void k_gather_kept(int64_t m, const uint32_t *__restrict__ rows,
                              const uint64_t *__restrict__ keys, const double *__restrict__ psi,
                              uint64_t *__restrict__ keys_t, double *__restrict__ psi_t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t r = rows[i];
    keys_t[i] = keys[r];
    psi_t[i] = psi[r];
}

__global__ __launch_bounds__(BS) void k_norm2(int64_t n, const double *__restrict__ v,
                                              double *__restrict__ partials) {
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n; r += (int64_t)gridDim.x * BS)
        acc += v[r] * v[r];
    store_partial<BS>(block_sum<BS>(acc), partials);
}

__global__ void k_scale_by(int64_t n, double *__restrict__ v, const double *__restrict__ nrm2) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    v[r] *= scale_from(nrm2, 1);
}

struct SelOps {
    int n;
    int orb[32];
    int spin[32];
};

// Jordan-Wigner sign of c+_{i s} / c_{i s} on (up, dn): electrons in the
// orbitals ordered before (i, s) with all up orbitals first.
__device__ __forceinline__ double jw_sign(uint32_t up, uint32_t dn, int i, int spin) {
    const uint32_t below = (1u << i) - 1u;
    const int par = spin == 0 ? __popc(up & below) : __popc(up) + __popc(dn & below);
    return (par & 1) ? -1.0 : 1.0;
}

__device__ __forceinline__ bool image(uint64_t key, int i, int spin, bool create, uint64_t *out) {
    const uint32_t up = (uint32_t)(key >> 32), dn = (uint32_t)key;
    const uint32_t s = spin == 0 ? up : dn;
    const bool occ = (s >> i) & 1u;
    if (occ == create) return false;
    *out = key ^ ((uint64_t)(1u << i) << (spin == 0 ? 32 : 0));
    return true;
}

__global__ void k_images(int64_t m, const uint64_t *__restrict__ keys, SelOps sel, int create,
                         uint64_t *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const uint64_t k = keys[r];
    for (int q = 0; q < sel.n; q++) {
        uint64_t t;
        out[r * sel.n + q] = image(k, sel.orb[q], sel.spin[q], create != 0, &t) ? t : kEmpty;
    }
}

template <typename T>
__global__ void k_start_block(int64_t m, const uint64_t *__restrict__ keys,
                              const double *__restrict__ psi, SelOps sel, int create,
                              const HashSlot *__restrict__ h, uint64_t hmask, int P,
                              T *__restrict__ phi) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const uint64_t k = keys[r];
    const uint32_t up = (uint32_t)(k >> 32), dn = (uint32_t)k;
    for (int q = 0; q < sel.n; q++) {
        uint64_t t;
        if (!image(k, sel.orb[q], sel.spin[q], create != 0, &t)) continue;
        const int64_t row = hash_find(h, hmask, t);
        if (row >= 0) phi[row * P + q] = (T)(jw_sign(up, dn, sel.orb[q], sel.spin[q]) * psi[r]);
    }
}

// Column k of a row-major [n][P] block to / from a contiguous vector
// (dir 0: v = B[:, k]; dir 1: B[:, k] = v).
template <typename T>
__global__ void k_column(int64_t n, int P, int k, T *__restrict__ B, T *__restrict__ v, int dir) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (dir == 0)
        v[r] = B[r * P + k];
    else
        B[r * P + k] = v[r];
}

// Partial Gram matrices: partial[(m * nch + chunk)][a][b] = sum over the
// chunk's rows of Q_m[r][a] X[r][b] (float64 accumulation, fixed order).
template <typename T, int P>
__global__ __launch_bounds__(BS) void k_gram(int64_t n, int64_t chunk_rows, int nch,
                                             const T *__restrict__ Q0, int64_t qstride,
                                             const T *__restrict__ X, double *__restrict__ part) {
    constexpr int PP = P * P;
    constexpr int S = BS / PP;
    constexpr int TR = 32;
    __shared__ double sQ[TR][P];
    __shared__ double sX[TR][P];
    __shared__ double red[BS];
    const int chunk = blockIdx.x, m = blockIdx.y;
    const T *__restrict__ Q = Q0 + (int64_t)m * qstride;
    const int t = threadIdx.x;
    const int pair = t % PP, slice = t / PP;
    const int a = pair / P, b = pair % P;
    const int64_t r0 = (int64_t)chunk * chunk_rows;
    const int64_t r1 = min(r0 + chunk_rows, n);
    double acc = 0.0;
    for (int64_t base = r0; base < r1; base += TR) {
        const int rows = (int)min((int64_t)TR, r1 - base);
        for (int e = t; e < TR * P; e += BS) {
            const int rr = e / P, cc = e % P;
            const bool ok = rr < rows;
            sQ[rr][cc] = ok ? (double)Q[(base + rr) * P + cc] : 0.0;
            sX[rr][cc] = ok ? (double)X[(base + rr) * P + cc] : 0.0;
        }
        __syncthreads();
        for (int rr = slice; rr < TR; rr += S) acc += sQ[rr][a] * sX[rr][b];
        __syncthreads();
    }
    red[t] = acc;
    __syncthreads();
    if (t < PP) {
        double s = 0.0;
        for (int q = 0; q < S; q++) s += red[t + q * PP];
        part[((int64_t)m * nch + chunk) * PP + t] = s;
    }
}

// Partial Gram matrices Q_m^T X (P = 8, 16) of one row chunk for the blocks
// m in [m0, m0 + mc), mc <= gram_blocks<T>(), on the float64 matrix cores.  One
// v_mfma_f64_16x16x4f64 takes A (16 x 4) and B (4 x 16) from one double per
// lane -- lane l gives A[l % 16][l / 16] and B[l / 16][l % 16] -- and lane l
// holds D[l / 16 + 4 e][l % 16], e < 4, of the running 16 x 16 sum (this
// result layout checked on gfx950).  Lane l loads value l of 64 consecutive
// values of Q_m and of X, i.e. row g + l / P, column l % P, of the 64 / P
// rows from g on:
//   P = 16: A[i][k] = Q[g + k][i], B[k][j] = X[g + k][j]: D = the four
//   rows' Q^T X;
//   P = 8: two rows per operand row, A[8 h + a][k] = Q[g + 2 k + h][a] and
//   likewise B: the diagonal 8 x 8 blocks of D (h = h') are the sums over
//   the group's even and odd rows, the rest mixes rows and is dropped.
// Wavefront w takes the row groups g = r0 + (64 / P) (w + 4 i), U groups at a
// time: the X rows are loaded once for all mc blocks, then each block's Q
// rows, then the products (rows past the chunk's end enter as zeros).  Each
// block's sums are added over the wavefronts (and the two halves at P = 8)
// in LDS in a fixed order and stored at partial[(m * nch + chunk)][a][b] as
// for k_gram.  Float64 accumulation (inputs converted exactly), in the same
// order whatever mc and U are, so deterministic and independent of how blocks
// are grouped.  Blocks per workgroup: 4 for float64 blocks (X loaded once for
// four blocks, U = 4: C3 Grams with two reorthogonalisation passes 1.03 ->
// 0.93 s), 1 for float32 (U = 8: 42-52 VGPRs and 8 wavefronts per SIMD; four
// blocks at 110 VGPRs were 3% slower there).
template <typename T>
__host__ __device__ constexpr int gram_blocks() {
    return sizeof(T) == 8 ? 4 : 1;
}

template <typename T, int P>
__device__ __forceinline__ void gram_mfma_unit(int64_t n, int64_t chunk_rows, int nch,
                                               const T *__restrict__ Q0, int64_t qstride, int m0,
                                               int mc, const T *__restrict__ X,
                                               double *__restrict__ part, int chunk) {
    static_assert(P == 8 || P == 16, "matrix-core Gram for P = 8, 16");
    using D4 = double __attribute__((ext_vector_type(4)));
    constexpr int MB = gram_blocks<T>(), U = MB == 1 ? 8 : 4, RG = 64 / P, PP = P * P;
    __shared__ double red[4][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lr = lane / P, lc = lane % P;
    const int64_t r0 = (int64_t)chunk * chunk_rows;
    const int64_t r1 = min(r0 + chunk_rows, n);
    const GPtr<const T> Qg = (GPtr<const T>)Q0, Xg = (GPtr<const T>)X;
    D4 acc[MB];
#pragma unroll
    for (int i = 0; i < MB; i++) acc[i] = D4{0.0, 0.0, 0.0, 0.0};
    for (int64_t g = r0 + RG * w; g < r1; g += 4 * RG * U) {   // uniform over the wavefront
        double b[U], a[MB][U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t r = g + 4 * RG * u + lr;
            const T xv = Xg[min(r, r1 - 1) * P + lc];
            b[u] = r < r1 ? (double)xv : 0.0;
        }
#pragma unroll
        for (int i = 0; i < MB; i++) {
            if (i < mc) {   // uniform over the workgroup
                const int64_t qo = (int64_t)(m0 + i) * qstride;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int64_t r = g + 4 * RG * u + lr;
                    const T qv = Qg[qo + min(r, r1 - 1) * P + lc];
                    a[i][u] = r < r1 ? (double)qv : 0.0;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < MB; i++)
            if (i < mc)
#pragma unroll
                for (int u = 0; u < U; u++)
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][u], b[u], acc[i], 0, 0, 0);
    }
    const GPtr<double> pg = (GPtr<double>)part;
#pragma unroll
    for (int i = 0; i < MB; i++) {
        if (i >= mc) break;   // uniform
        if constexpr (P == 16) {
#pragma unroll
            for (int e = 0; e < 4; e++) red[w][((lane >> 4) + 4 * e) * 16 + (lane & 15)] = acc[i][e];
        } else {
            // rows < 8 for e < 2: columns < 8 keep e = 0, 1 (even rows),
            // columns >= 8 keep e = 2, 3 (odd rows)
            const int j = lane & 15, hh = j >> 3;
#pragma unroll
            for (int e = 0; e < 2; e++)
                red[w][64 * hh + ((lane >> 4) + 4 * e) * 8 + (j & 7)] = acc[i][2 * hh + e];
        }
        __syncthreads();
        if (t < PP) {
            double v;
            if constexpr (P == 16)
                v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
            else
                v = ((red[0][t] + red[0][64 + t]) + (red[1][t] + red[1][64 + t])) +
                    ((red[2][t] + red[2][64 + t]) + (red[3][t] + red[3][64 + t]));
            pg[((int64_t)(m0 + i) * nch + chunk) * PP + t] = v;
        }
        __syncthreads();
    }
}

// Partial Gram matrices Q_m^T X, m < nm, P = 8, 16: one dimension of 8
// ceil(nch / 8) ceil(nm / gram_blocks) workgroups, handed out XCD-major: the
// workgroups of one row chunk run on one XCD, so that the chunk's X rows are
// fetched once into its L2, and each loads them once for its blocks.
template <typename T, int P>
__global__ __launch_bounds__(256) void k_gram_rt(int64_t n, int64_t chunk_rows, int nch, int nm,
                                                 const T *__restrict__ Q0, int64_t qstride,
                                                 const T *__restrict__ X,
                                                 double *__restrict__ part) {
    constexpr int MB = gram_blocks<T>();
    const int nmg = (nm + MB - 1) / MB;
    const int k = blockIdx.x / 8, mg = k % nmg, chunk = (k / nmg) * 8 + blockIdx.x % 8;
    if (chunk >= nch) return;   // whole workgroup, before any barrier
    const int m0 = mg * MB;
    gram_mfma_unit<T, P>(n, chunk_rows, nch, Q0, qstride, m0, min(MB, nm - m0), X, part, chunk);
}

// out[m][e] = sum_c part[(m nch + c)][e]: one wavefront per output entry,
// lanes stride over the chunks, fixed butterfly order.
__device__ __forceinline__ void gram_reduce_wave(int nch, int PP, const double *__restrict__ part,
                                                 double *__restrict__ out, int i, int lane) {
    const int m = i / PP, e = i % PP;
    const double *__restrict__ pm = part + (int64_t)m * nch * PP + e;
    double s = 0.0;
    int c = lane;
    // eight loads in flight, then added in chunk order
    for (; c + 7 * 64 < nch; c += 8 * 64) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = pm[(int64_t)(c + u * 64) * PP];
#pragma unroll
        for (int u = 0; u < 8; u++) s += v[u];
    }
    for (; c < nch; c += 64) s += pm[(int64_t)c * PP];
    s = wave_sum(s);
    if (lane == 0) out[i] = s;
}

__global__ __launch_bounds__(256) void k_gram_reduce(int nm, int nch, int PP,
                                                     const double *__restrict__ part,
                                                     double *__restrict__ out) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nm * PP) return;          // whole wavefront exits together
    gram_reduce_wave(nch, PP, part, out, i, lane);
}

// W -= sum_{m < nm} Q_m C_m  (sub != 0)   or   W = Q_0 C_0  (sub == 0, nm == 1).
// C: nm float64 P x P matrices (row a, column b), kept in LDS.
template <typename T, int P>
__global__ __launch_bounds__(BS) void k_block_apply(int64_t n, int nm, const T *__restrict__ Q0,
                                                    int64_t qstride, const double *__restrict__ C,
                                                    T *__restrict__ W, int sub) {
    constexpr int RPB = BS / P;
    extern __shared__ double sC[];
    for (int e = threadIdx.x; e < nm * P * P; e += BS) sC[e] = C[e];
    __syncthreads();
    const int b = threadIdx.x % P;
    for (int64_t tile = blockIdx.x; tile * RPB < n; tile += gridDim.x) {
        const int64_t r = tile * RPB + threadIdx.x / P;
        if (r >= n) continue;
        double acc = 0.0;
        for (int m = 0; m < nm; m++) {
            const T *__restrict__ q = Q0 + (int64_t)m * qstride + r * P;
            const double *__restrict__ c = sC + m * P * P;
#pragma unroll
            for (int a = 0; a < P; a++) acc += (double)q[a] * c[a * P + b];
        }
        if (sub)
            W[r * P + b] = (T)((double)W[r * P + b] - acc);
        else
            W[r * P + b] = (T)acc;
    }
}

// k_block_apply with one thread per row (P >= 4): row r of W (-)= sum_m
// Q_m C_m.  The row's P values of each block come in 16-byte loads and are
// converted once, the P outputs are accumulated in registers; each output
// receives the same terms in the same (m, a) order as k_block_apply, so the
// results are bit-identical.  The blocks are read as global memory (generic
// pointers, as taken from a run table, would otherwise make flat loads that
// wait together with everything else), and the coefficients C (read-only,
// the same for the whole workgroup) through the constant address space, so
// they arrive by scalar loads and feed the multiply-adds from scalar
// registers (no LDS copy, no per-lane loads).
template <typename T, int P>
__device__ __forceinline__ void block_apply_row(int64_t r, int nm, const T *Q0p, int64_t qstride,
                                                const double *__restrict__ C, T *Wp, int sub) {
    constexpr int U = 16 / sizeof(T);
    using V16 = T __attribute__((ext_vector_type(16 / sizeof(T))));
    const GPtr<const T> Q0 = (GPtr<const T>)Q0p;
    const GPtr<T> W = (GPtr<T>)Wp;
    double acc[P];
#pragma unroll
    for (int b = 0; b < P; b++) acc[b] = 0.0;
    for (int m = 0; m < nm; m++) {
        const GPtr<const V16> q = (GPtr<const V16>)(Q0 + (int64_t)m * qstride + r * P);
        V16 qv[P / U];
#pragma unroll
        for (int u = 0; u < P / U; u++) qv[u] = q[u];
        // read-only for the kernel and the same for the whole workgroup:
        // through the constant address space, so they come by scalar loads
        const __attribute__((address_space(4))) double *c =
            (const __attribute__((address_space(4))) double *)(C + m * P * P);
#pragma unroll
        for (int a = 0; a < P; a++) {
            const double qa = (double)qv[a / U][a % U];
#pragma unroll
            for (int b = 0; b < P; b++) acc[b] += qa * c[a * P + b];
        }
    }
    const GPtr<V16> w = (GPtr<V16>)(W + r * P);
#pragma unroll
    for (int u = 0; u < P / U; u++) {
        V16 o;
        if (sub) {
            const V16 wv = w[u];
#pragma unroll
            for (int e = 0; e < U; e++) o[e] = (T)((double)wv[e] - acc[u * U + e]);
        } else {
#pragma unroll
            for (int e = 0; e < U; e++) o[e] = (T)acc[u * U + e];
        }
        w[u] = o;
    }
}

template <typename T, int P>
__global__ __launch_bounds__(BS) void k_block_apply_r(int64_t n, int nm, const T *__restrict__ Q0,
                                                      int64_t qstride, const double *__restrict__ C,
                                                      T *__restrict__ W, int sub) {
    static_assert(P * sizeof(T) % 16 == 0, "row of P values must be whole 16-byte units");
    for (int64_t r = (int64_t)blockIdx.x * BS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * BS)
        block_apply_row<T, P>(r, nm, Q0, qstride, C, W, sub);
}

// W (-)= sum_m Q_m C_m for nm blocks (C on the device), one launch; block m
// at Q0 + m qstride (elements; negative where a ring of blocks wraps).
template <typename T, int P>
static void launch_block_apply(int64_t n, int nm, const T *Q0, int64_t qstride, const double *C,
                               T *W, bool sub, hipStream_t s) {
    const size_t lds = (size_t)nm * P * P * sizeof(double);
    if constexpr (P * sizeof(T) % 16 == 0) {
        const unsigned nb = (unsigned)std::min<int64_t>(gridn(n, BS), 8192);
        hipLaunchKernelGGL((k_block_apply_r<T, P>), dim3(nb), dim3(BS), 0, s, n, nm, Q0, qstride,
                           C, W, sub ? 1 : 0);
    } else {
        const unsigned nb = (unsigned)std::min<int64_t>(gridn(n, BS / P), 4096);
        hipLaunchKernelGGL((k_block_apply<T, P>), dim3(nb), dim3(BS), lds, s, n, nm, Q0,
                           qstride, C, W, sub ? 1 : 0);
    }
}

// ---------------------------------------------------------------------------
// Host small linear algebra (float64 / complex128, P <= 16).
// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major):
// A = V diag(w) V^T, columns of V are eigenvectors.
static void jacobi_eig(int n, std::vector<double> A, std::vector<double> &w,
                       std::vector<double> &V) {
    V.assign(n * n, 0.0);
    for (int i = 0; i < n; i++) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                (i == j ? diag : off) += A[i * n + j] * A[i * n + j];
        if (off <= 1e-30 * std::max(diag, 1e-300)) break;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) {
                const double apq = A[p * n + q];
                if (fabs(apq) < 1e-300) continue;
                // rotation angle that zeroes A[p][q]
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                for (int k = 0; k < n; k++) {   // columns p, q
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {   // rows p, q
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; i++) w[i] = A[i * n + i];
}

// Host worker pool for the small dense host work (block continued fractions,
// per-frequency solves): up to 15 workers beside the calling thread, created
// on first use and kept for the life of the process (the pool object is
// never destroyed, so no worker is joined at exit; idle workers wait on a
// condition variable).  One loop at a time: a call that finds the pool busy
// (another host thread, or a call from inside a loop) runs in the calling
// thread alone.
class HostPool {
  public:
    static HostPool &get() {
        static HostPool *p = new HostPool();
        return *p;
    }
    int workers() const { return nworkers_; }
    // fn(i) for every i in [0, n), the items handed out one at a time;
    // false (nothing run) when the pool is busy
    bool run(int n, const std::function<void(int)> &fn) {
        std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
        if (!busy.owns_lock()) return false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &fn;
            total_ = n;
            next_.store(0);
            pending_ = nworkers_;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return pending_ == 0; });   // no worker still reads fn
        job_ = nullptr;
        return true;
    }

  private:
    HostPool() {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        nworkers_ = std::max(0, std::min(hw, 16) - 1);
        for (int t = 0; t < nworkers_; t++) std::thread([this] { loop(); }).detach();
    }
    void work() {
        for (int i = next_.fetch_add(1); i < total_; i = next_.fetch_add(1)) (*job_)(i);
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
            }
            work();
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_cv_.notify_one();
        }
    }
    std::mutex run_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *job_ = nullptr;
    int total_ = 0, nworkers_ = 0, pending_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
};

// fn(i) for i in [0, n) on the host pool (or in the calling thread); the
// callers give every index its own output, so results do not depend on
// which thread ran which index.
template <typename F>
static void parallel_for(int n, F &&fn) {
    if (n <= 0) return;
    if (n > 1 && HostPool::get().workers() > 0) {
        const std::function<void(int)> f = [&](int i) { fn(i); };
        if (HostPool::get().run(n, f)) return;
    }
    for (int i = 0; i < n; i++) fn(i);
}

// Solve S X = B for complex S (n x n) and B (n x k), row-major, real and
// imaginary parts in separate arrays, by Gaussian elimination with partial
// pivoting (pivot: largest |S_rc|^2 in the column); S and B are overwritten,
// X returned in B.  Complex products are written out and each pivot is
// inverted once (scaled by its larger component), so no library complex
// division or multiplication with its special-value handling is called.
static void csolve_split(int n, int k, double *Sr, double *Si, double *Br, double *Bi) {
    auto inv = [](double a, double b, double &ir, double &ii) {
        const double sc = std::max(std::fabs(a), std::fabs(b));
        const double as = a / sc, bs = b / sc;
        const double den = sc * (as * as + bs * bs);
        ir = as / den;
        ii = -bs / den;
    };
    for (int c = 0; c < n; c++) {
        int piv = c;
        double best = Sr[c * n + c] * Sr[c * n + c] + Si[c * n + c] * Si[c * n + c];
        for (int r = c + 1; r < n; r++) {
            const double v = Sr[r * n + c] * Sr[r * n + c] + Si[r * n + c] * Si[r * n + c];
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (piv != c) {
            for (int j = c; j < n; j++) {
                std::swap(Sr[c * n + j], Sr[piv * n + j]);
                std::swap(Si[c * n + j], Si[piv * n + j]);
            }
            for (int j = 0; j < k; j++) {
                std::swap(Br[c * k + j], Br[piv * k + j]);
                std::swap(Bi[c * k + j], Bi[piv * k + j]);
            }
        }
        double dr, di;
        inv(Sr[c * n + c], Si[c * n + c], dr, di);
        for (int r = c + 1; r < n; r++) {
            const double ar = Sr[r * n + c], ai = Si[r * n + c];
            const double fr = ar * dr - ai * di, fi = ar * di + ai * dr;
            if (fr == 0.0 && fi == 0.0) continue;
            for (int j = c + 1; j < n; j++) {
                const double ur = Sr[c * n + j], ui = Si[c * n + j];
                Sr[r * n + j] -= fr * ur - fi * ui;
                Si[r * n + j] -= fr * ui + fi * ur;
            }
            for (int j = 0; j < k; j++) {
                const double ur = Br[c * k + j], ui = Bi[c * k + j];
                Br[r * k + j] -= fr * ur - fi * ui;
                Bi[r * k + j] -= fr * ui + fi * ur;
            }
        }
    }
    for (int c = n - 1; c >= 0; c--) {
        double dr, di;
        inv(Sr[c * n + c], Si[c * n + c], dr, di);
        for (int j = 0; j < k; j++) {
            double sr = Br[c * k + j], si = Bi[c * k + j];
            for (int q = c + 1; q < n; q++) {
                const double ar = Sr[c * n + q], ai = Si[c * n + q];
                const double xr = Br[q * k + j], xi = Bi[q * k + j];
                sr -= ar * xr - ai * xi;
                si -= ar * xi + ai * xr;
            }
            Br[c * k + j] = sr * dr - si * di;
            Bi[c * k + j] = sr * di + si * dr;
        }
    }
}

// The same solve on interleaved complex vectors.
static void csolve(int n, int k, std::vector<cplx> &S, std::vector<cplx> &B) {
    std::vector<double> Sr(n * n), Si(n * n), Br(n * k), Bi(n * k);
    for (int e = 0; e < n * n; e++) {
        Sr[e] = S[e].real();
        Si[e] = S[e].imag();
    }
    for (int e = 0; e < n * k; e++) {
        Br[e] = B[e].real();
        Bi[e] = B[e].imag();
    }
    csolve_split(n, k, Sr.data(), Si.data(), Br.data(), Bi.data());
    for (int e = 0; e < n * k; e++) B[e] = cplx(Br[e], Bi[e]);
}

struct BandResult {
    std::vector<std::vector<double>> A;   // A_j, P x P
    std::vector<std::vector<double>> B;   // B_j (j >= 1), P x P; B[0] unused
    std::vector<double> R0;               // P x P: start block = Q_0 R0
    int P = 0;
    int m = 0;                            // number of blocks in T
    int krylov = 0;                       // nonzero Lanczos directions
};

// G_sub(z) = R0^T [(z - T)^-1]_00 R0 for one z; out p x p (first p columns).
// The block continued fraction from the last block up: S_{m-1} = z - A_{m-1},
// S_j = z - A_j - B_{j+1}^T S_{j+1}^-1 B_{j+1}; then R0^T S_0^-1 R0.  P <= 16;
// no heap allocation (it runs at every convergence check).
static void block_cf(const BandResult &br, cplx z, int p, cplx *out) {
    constexpr int kMax = 16;
    const int P = br.P, m = br.m;
    if (m <= 0 || P <= 0 || P > kMax) {
        for (int e = 0; e < p * p; e++) out[e] = 0.0;
        return;
    }
    double Sr[kMax * kMax], Si[kMax * kMax], Xr[kMax * kMax], Xi[kMax * kMax];
    const double zr = z.real(), zi = z.imag();
    auto zA = [&](int j) {
        const double *A = br.A[j].data();
        for (int a = 0; a < P; a++)
            for (int b = 0; b < P; b++) {
                Sr[a * P + b] = (a == b ? zr : 0.0) - A[a * P + b];
                Si[a * P + b] = a == b ? zi : 0.0;
            }
    };
    zA(m - 1);
    for (int j = m - 2; j >= 0; j--) {
        // X = S^-1 B_{j+1};  S_j = z - A_j - B_{j+1}^T X
        const double *Bj = br.B[j + 1].data();
        for (int e = 0; e < P * P; e++) {
            Xr[e] = Bj[e];
            Xi[e] = 0.0;
        }
        csolve_split(P, P, Sr, Si, Xr, Xi);
        zA(j);
        for (int a = 0; a < P; a++)
            for (int b = 0; b < P; b++) {
                double sr = 0.0, si = 0.0;
                for (int q = 0; q < P; q++) {
                    const double bq = Bj[q * P + a];
                    sr += bq * Xr[q * P + b];
                    si += bq * Xi[q * P + b];
                }
                Sr[a * P + b] -= sr;
                Si[a * P + b] -= si;
            }
    }
    const double *R0 = br.R0.data();
    for (int e = 0; e < P * P; e++) {
        Xr[e] = R0[e];
        Xi[e] = 0.0;
    }
    csolve_split(P, P, Sr, Si, Xr, Xi);
    for (int a = 0; a < p; a++)
        for (int b = 0; b < p; b++) {
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < P; q++) {
                sr += R0[q * P + a] * Xr[q * P + b];
                si += R0[q * P + a] * Xi[q * P + b];
            }
            out[a * p + b] = cplx(sr, si);
        }
}

// ---------------------------------------------------------------------------
// Small dense steps of the block recurrence on the device (P <= 16, one
// workgroup of one wavefront): the coefficient matrices never leave HBM, so
// a block step needs no host round trip.

// Coefficients of W -= Q_{j-1} B_j^T + Q_j A_j in one pass over W:
// A_j = sym(G) (also kept in dA), C2 = [B_j^T ; A_j] (B_j^T only when dB).
__device__ __forceinline__ void sym_pair_body(int P, const double *__restrict__ G,
                                              double *__restrict__ dA,
                                              const double *__restrict__ dB,
                                              double *__restrict__ C2) {
    const int PP = P * P;
    for (int e = threadIdx.x; e < PP; e += 64) {
        const int a = e / P, b = e % P;
        const double v = 0.5 * (G[a * P + b] + G[b * P + a]);
        dA[e] = v;
        C2[PP + e] = v;
        if (dB != nullptr) C2[e] = dB[b * P + a];
    }
}

__global__ __launch_bounds__(64) void k_sym_pair(int P, const double *__restrict__ G,
                                                 double *__restrict__ dA,
                                                 const double *__restrict__ dB,
                                                 double *__restrict__ C2) {
    sym_pair_body(P, G, dA, dB, C2);
}

// QR factor of a block W from its Gram matrix M = W^T W by pivoted Cholesky
// (rank revealing, the band method's deflation): at step k the column with
// the largest remaining Schur diagonal d is taken if d > thr (thr = thr_abs
// for mode 0, 1e-2 max diag M for mode 1, the re-orthogonalising pass), row k
// of R = sqrt(d)^-1 (Schur row), and the Schur complement is updated.  With
// rank r, W = Q R (R: r x P, zero rows below), Q = W Xm with
// Xm = Pi R11^-1 (zero columns beyond r).  Bacc <- R Bacc (R itself when
// init; Bacc's rows past the previous rank are zero), *rank_out = r.
// One wavefront, P a compile-time power of two: every loop is unrolled, the
// chosen set is a register mask (the same in every lane), and M and Bacc are
// loaded together at the start, so the steps are LDS round trips only.
template <int P>
__device__ __forceinline__ void pchol_body(const double *__restrict__ M, int mode,
                                           double thr_abs, double *__restrict__ Xm,
                                           double *__restrict__ Bm, double *__restrict__ Bacc,
                                           int init, int *__restrict__ rank_out) {
    constexpr int PP = P * P;
    __shared__ double S[P][P], R[P][P], Ri[P][P], U[P][P], Bs[P][P];
    __shared__ int piv[P];
    const int t = threadIdx.x;
    for (int e = t; e < PP; e += 64) {
        const int a = e / P, b = e % P;
        S[a][b] = M[e];
        Bs[a][b] = init ? 0.0 : Bacc[e];
        R[a][b] = 0.0;
        Ri[a][b] = 0.0;
    }
    if (t < P) piv[t] = 0;
    __syncthreads();
    double maxd = 0.0;
#pragma unroll
    for (int i = 0; i < P; i++) maxd = fmax(maxd, S[i][i]);
    const double thr = mode == 0 ? thr_abs : 1e-2 * maxd;
    unsigned chosen = 0u;
    int r = 0;
#pragma unroll
    for (int k = 0; k < P; k++) {
        double d[P];
#pragma unroll
        for (int i = 0; i < P; i++) d[i] = S[i][i];
        int q = -1;
        double dq = 0.0;
#pragma unroll
        for (int i = 0; i < P; i++)
            if (!((chosen >> i) & 1u) && d[i] > dq) {
                dq = d[i];
                q = i;
            }
        if (q < 0 || !(dq > thr)) break;     // the same decision in every lane
        const double sq = sqrt(dq);
        if (t < P) R[k][t] = ((chosen >> t) & 1u) ? 0.0 : S[q][t] / sq;
        __syncthreads();
        chosen |= 1u << q;
        if (t == 0) piv[k] = q;
        for (int e = t; e < PP; e += 64) {
            const int i = e / P, j = e % P;
            S[i][j] -= R[k][i] * R[k][j];
        }
        __syncthreads();
        r++;
    }
    // R11 with its columns in pivot order: U[k][m] = R[k][piv[m]]
    for (int e = t; e < PP; e += 64) {
        const int k = e / P, m = e % P;
        U[k][m] = m < r ? R[k][piv[m]] : 0.0;
    }
    __syncthreads();
    // R11^-1 (upper triangular), one column l per lane, back substitution
    // from the diagonal up, each entry summed in ascending order
    if (t < r) {
        const int l = t;
        double x[P];
#pragma unroll
        for (int kk = P - 1; kk >= 0; kk--) {
            x[kk] = 0.0;
            if (kk == l) {
                x[kk] = 1.0 / U[l][l];
            } else if (kk < l) {
                double acc = 0.0;
#pragma unroll
                for (int mm = kk + 1; mm < P; mm++)
                    if (mm <= l) acc += U[kk][mm] * x[mm];
                x[kk] = -acc / U[kk][kk];
            }
        }
#pragma unroll
        for (int kk = 0; kk < P; kk++)
            if (kk <= l) Ri[kk][l] = x[kk];
    }
    __syncthreads();
    for (int e = t; e < PP; e += 64) {
        const int a = e / P, c = e % P;   // Xm row a (column of W), column c (new direction)
        double x = 0.0;
#pragma unroll
        for (int l = 0; l < P; l++)
            if (l <= c && c < r && piv[l] == a) x = Ri[l][c];
        Xm[e] = x;
        Bm[e] = a < r ? R[a][c] : 0.0;    // Bm row a, column c
        // Bacc <- R Bacc (the previous Bacc is in Bs)
        double acc = 0.0;
        if (init) {
            acc = a < r ? R[a][c] : 0.0;
        } else if (a < r) {
#pragma unroll
            for (int q = 0; q < P; q++) acc += R[a][q] * Bs[q][c];
        }
        Bacc[e] = acc;
    }
    if (t == 0) *rank_out = r;
}

template <int P>
__global__ __launch_bounds__(64) void k_pchol(const double *__restrict__ M, int mode,
                                              double thr_abs, double *__restrict__ Xm,
                                              double *__restrict__ Bm,
                                              double *__restrict__ Bacc, int init,
                                              int *__restrict__ rank_out) {
    pchol_body<P>(M, mode, thr_abs, Xm, Bm, Bacc, init, rank_out);
}

// Frequency argument zeta of G: i w (Matsubara, eta <= 0) or w + i eta
// (real frequency, Lorentzian width eta).  G+ is evaluated at z = E0 + zeta
// and G- at z = E0 - zeta.
static inline cplx freq_arg(const mcd_band_cfg *cfg, double w) {
    return cfg->eta > 0.0 ? cplx(w, cfg->eta) : cplx(0.0, w);
}

static double wall_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---------------------------------------------------------------------------
// One band run: block Lanczos on one excited sector (F~+ or F~-) of one
// instance.  Every buffer is a piece of the caller's workspace.  The device
// form keeps the whole recurrence on the GPU (Gram matrices, coefficients,
// pivoted-Cholesky QR); several runs advance in lockstep (run_lockstep), so
// the particle and hole runs of one call, and the runs of many instances,
// share every block step on one stream.
template <typename T>
struct BandRun {
    const mcd_op *op = nullptr;   // operator on F~+- (owned: destroyed in release())
    int P = 0;
    int64_t n = 0;
    hipStream_t s = nullptr;
    int mb = 0;                   // max block steps
    int limit = 0;                // > 0: stop after this many block steps (a replay)
    int nstore = 0;               // stored blocks: mb + 1, or a ring of 3
    T *Qs = nullptr;              // [nstore][n][P]
    T *W = nullptr;               // [n][P]
    T *W2 = nullptr;              // [n][P] scratch of the two-pass QR (device form)
    T *colbuf = nullptr;          // [2][n] single-column staging (per-column form)
    bool per_column = false;
    double *part = nullptr;       // Gram partials
    int64_t part_cap = 0;
    double *dG = nullptr;         // reduced Gram matrices [(mb + 1) P P]
    double *dC = nullptr;         // coefficients staged from the host [(mb + 1) P P]
    double *dT = nullptr;         // [A: mb][B: mb + 1][R0][Xm][Bm][Bacc][C2: 2], P x P each
    int *d_rank = nullptr;        // [mb + 2]
    int64_t chunk_rows = 0;       // Gram row chunks (fixed per run)
    int nch = 0;
    Alloc al;
    std::vector<void *> pieces;   // workspace pieces of the run (released together)
    // lockstep state
    bool active = false;
    int m = 0;                    // block steps in T
    std::vector<int> rank;        // host copy of d_rank
    std::vector<double> hT;       // host copy of dT
    BandResult br;
    // convergence of G: stop when G at the check points zcheck changes by
    // <= g_tol max|G| between two checks (8 block steps apart)
    std::vector<cplx> zcheck;
    double g_tol = 0.0;
    int p_sel = 1;
    std::vector<cplx> gprev;

    BandRun() = default;
    BandRun(const BandRun &) = delete;
    BandRun &operator=(const BandRun &) = delete;
    ~BandRun() { release(); }

    int PP() const { return P * P; }
    T *blk(int j) { return Qs + (int64_t)(nstore == 3 ? j % 3 : j) * n * P; }
    double *dA(int j) { return dT + (size_t)j * PP(); }
    double *dB(int j) { return dT + (size_t)(mb + j) * PP(); }
    double *dR0() { return dT + (size_t)(2 * mb + 1) * PP(); }
    double *dXm() { return dR0() + PP(); }
    double *dBm() { return dXm() + PP(); }
    double *dBacc() { return dBm() + PP(); }
    double *dC2() { return dBacc() + PP(); }
    size_t nT() const { return (size_t)(2 * mb + 7) * PP(); }

    // the run's pieces back to the workspace, its operator destroyed
    void release() {
        if (op) mcd_op_destroy(const_cast<mcd_op *>(op));
        op = nullptr;
        for (auto it = pieces.rbegin(); it != pieces.rend(); ++it) (void)dfree(*it, al);
        pieces.clear();
        Qs = W = W2 = colbuf = nullptr;
        part = dG = dC = dT = nullptr;
        d_rank = nullptr;
    }
    hipError_t take(void **p, size_t bytes) {
        const hipError_t e = dmalloc(p, bytes, al);
        if (e == hipSuccess) pieces.push_back(*p);
        return e;
    }

    // Gram row chunks of the run: a function of (n, P, T) only, so a run
    // gives the same sums whichever runs share its launches.  Matrix-core
    // kernels (P >= 8): at least 8 rpb rows per chunk (rpb = 256, 128 or 64
    // for float32 P = 8, float64 P = 8 and P = 16) and at most 1024 chunks;
    // LDS kernel (P < 8): at least 256 rows per chunk, at most 2048 chunks.
    void set_chunks() {
        int64_t c;
        if (P >= 8) {
            const int64_t rpb = 256 / (P == 16 ? 4 : sizeof(T) == 8 ? 2 : 1);
            c = std::max<int64_t>(1, std::min<int64_t>(n / (8 * rpb), 1024));
            if (c > 8) c = (c + 7) / 8 * 8;
        } else {
            c = std::min<int64_t>(gridn(n, 256), 2048);
        }
        c = std::max<int64_t>(1, c);
        // an empty sector (n = 0) has one empty chunk size and no chunks
        chunk_rows = std::max<int64_t>(1, (n + c - 1) / c);
        nch = (int)((n + chunk_rows - 1) / chunk_rows);
    }
    // Gram partial capacity for up to mb + 1 blocks at once
    int64_t partials_needed() const {
        const int64_t pad = P >= 8 ? ((int64_t)nch + 7) / 8 * 8 : nch;
        return pad * (int64_t)(mb + 1) * PP();
    }

    // G at the check points is wanted for this T
    bool g_wanted(const BandResult &b) const { return g_tol > 0.0 && !zcheck.empty() && b.m > 0; }
    // G at the check points (zcheck.size() blocks of p_sel x p_sel, from
    // block_cf) against the previous check's: settled when the largest change
    // is within g_tol of the largest |G|; g becomes the previous values
    bool g_settled(std::vector<cplx> &&g) {
        bool conv = false;
        if (gprev.size() == g.size()) {
            double dmax = 0.0, gmax = 0.0;
            for (size_t e = 0; e < g.size(); e++) {
                dmax = std::max(dmax, std::abs(g[e] - gprev[e]));
                gmax = std::max(gmax, std::abs(g[e]));
            }
            conv = dmax <= g_tol * gmax;
        }
        gprev = std::move(g);
        return conv;
    }
    bool g_converged(const BandResult &b) {
        if (!g_wanted(b)) return false;
        std::vector<cplx> g((size_t)zcheck.size() * p_sel * p_sel);
        parallel_for((int)zcheck.size(), [&](int f) {
            block_cf(b, zcheck[f], p_sel, g.data() + (size_t)f * p_sel * p_sel);
        });
        return g_settled(std::move(g));
    }

    int gram(const T *Q0, int nm, const T *X, std::vector<double> &out) {
        const int PP = P * P;
        MCD_TRY(gram_dev(Q0, nm, X));
        out.resize((size_t)nm * PP);
        MCD_HIP(hipMemcpyAsync(out.data(), dG, (size_t)nm * PP * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        MCD_HIP(hipStreamSynchronize(s));
        return MCD_OK;
    }

    // Gram matrices Q_m^T X (m < nm) into dG on the device.
    int gram_dev(const T *Q0, int nm, const T *X) {
        const int PP = P * P;
        MCD_REQUIRE((int64_t)nm * (P >= 8 ? ((int64_t)nch + 7) / 8 * 8 : nch) * PP <= part_cap,
                    MCD_E_CAPACITY, "gram scratch too small");
        dim3 grid(nch, nm);
#define GR(PV)                                                                           \
    case PV:                                                                             \
        hipLaunchKernelGGL((k_gram<T, PV>), grid, dim3(BS), 0, s, n, chunk_rows, nch, Q0, \
                           (int64_t)n * P, X, part);                                     \
        break;
#define GRT(PV)                                                                              \
    case PV:                                                                                 \
        hipLaunchKernelGGL((k_gram_rt<T, PV>),                                                 \
                           dim3((unsigned)((nch + 7) / 8 * 8 *                               \
                                           ((nm + gram_blocks<T>() - 1) / gram_blocks<T>()))), \
                           dim3(256), 0, s, n, chunk_rows, nch, nm, Q0, (int64_t)n * P, X,   \
                           part);                                                            \
        break;
        switch (P) {
            GR(1) GR(2) GR(4) GRT(8) GRT(16)
        }
#undef GR
#undef GRT
        MCD_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_gram_reduce, dim3(gridn((int64_t)nm * PP, 4)), dim3(256), 0, s, nm,
                           nch, PP, part, dG);
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    }

    // W (-)= sum_m Q_m C_m with C already on the device ([nm][P][P]); block m
    // at Q0 + m qstride (0: consecutive blocks of the store).
    int block_apply_dev(const T *Q0, int nm, const double *C, T *Wout, bool sub,
                        int64_t qstride = 0) {
        const int PP = P * P;
        const int group = std::max(1, (48 * 1024) / (PP * 8));
        MCD_REQUIRE(sub || nm <= group, MCD_E_INVALID, "assigning block product must use one group");
        if (qstride == 0) qstride = (int64_t)n * P;
        for (int g0 = 0; g0 < nm; g0 += group) {
            const int g = std::min(group, nm - g0);
            const T *q = Q0 + (int64_t)g0 * qstride;
            const double *c = C + (size_t)g0 * PP;
#define BAD(PV)                                                     \
    case PV:                                                        \
        launch_block_apply<T, PV>(n, g, q, qstride, c, Wout, sub, s); \
        break;
            switch (P) {
                BAD(1) BAD(2) BAD(4) BAD(8) BAD(16)
            }
#undef BAD
            MCD_HIP(hipGetLastError());
        }
        return MCD_OK;
    }

    // W (-)= sum_m Q_m C_m with C given on the host ([nm][P][P]); the staging
    // buffer dC holds every group at once, so no copy overwrites coefficients
    // a queued product still reads.
    int block_apply(const T *Q0, int nm, const std::vector<double> &C, T *Wout, bool sub) {
        const int PP = P * P;
        MCD_REQUIRE((size_t)nm * PP <= (size_t)(mb + 1) * PP, MCD_E_CAPACITY,
                    "coefficient staging too small");
        MCD_REQUIRE(sub || nm <= std::max(1, (48 * 1024) / (PP * 8)), MCD_E_INVALID,
                    "assigning block product must use one group");
        MCD_HIP(hipMemcpyAsync(dC, C.data(), (size_t)nm * PP * sizeof(double),
                               hipMemcpyHostToDevice, s));
        MCD_TRY(block_apply_dev(Q0, nm, dC, Wout, sub));
        MCD_HIP(hipStreamSynchronize(s));   // C (host) is read by the copy above
        return MCD_OK;
    }

    // Orthonormalise X (n x P) into dst: X = dst Bout; drops directions with
    // Gram eigenvalue <= thr2 (first pass) and repeats once for accuracy.
    int qr(T *X, T *dst, double thr2, std::vector<double> &Bout, int *rank_out) {
        const int PP = P * P;
        std::vector<double> Bacc(PP, 0.0);
        for (int i = 0; i < P; i++) Bacc[i * P + i] = 1.0;
        T *src = X;
        for (int pass = 0; pass < 2; pass++) {
            std::vector<double> M, w, V;
            MCD_TRY(gram(src, 1, src, M));
            for (double v : M)
                MCD_REQUIRE(std::isfinite(v), MCD_E_NUMERIC,
                            "band Lanczos: non-finite Gram matrix (NaN or Inf in psi0 or H)");
            jacobi_eig(P, M, w, V);
            std::vector<double> Xm(PP, 0.0), Bm(PP, 0.0);
            double wmax = 0.0;
            for (int i = 0; i < P; i++) wmax = std::max(wmax, w[i]);
            const double th = pass == 0 ? thr2 : 1e-2 * std::max(wmax, 1e-300);
            int rk = 0;
            for (int i = 0; i < P; i++) {
                if (w[i] <= th || w[i] <= 0.0) continue;
                rk++;
                const double sq = sqrt(w[i]);
                for (int a = 0; a < P; a++) {
                    Xm[a * P + i] = V[a * P + i] / sq;   // column i of U L^-1/2
                    Bm[i * P + a] = sq * V[a * P + i];   // row i of L^1/2 U^T
                }
            }
            *rank_out = rk;
            // dst = src Xm  (when src == dst go through W)
            T *out = (src == dst) ? W : dst;
            MCD_TRY(block_apply(src, 1, Xm, out, false));
            if (out != dst)
                MCD_HIP(hipMemcpyAsync(dst, out, (size_t)n * P * sizeof(T), hipMemcpyDeviceToDevice,
                                       s));
            // Bacc = Bm Bacc
            std::vector<double> nb(PP, 0.0);
            for (int i = 0; i < P; i++)
                for (int j = 0; j < P; j++) {
                    double acc = 0.0;
                    for (int q = 0; q < P; q++) acc += Bm[i * P + q] * Bacc[q * P + j];
                    nb[i * P + j] = acc;
                }
            Bacc = nb;
            src = dst;
            if (rk == 0) break;
        }
        Bout = Bacc;
        return MCD_OK;
    }

    // Device QR of src into dst (two pivoted-Cholesky passes through W2); the
    // factor goes to outB, the rank to d_rank[slot].  src and dst are never W2.
    int qr_dev(T *src, T *dst, double *outB, int slot, double dtol_abs) {
        T *cur = src;
        for (int pass = 0; pass < 2; pass++) {
            MCD_TRY(gram_dev(cur, 1, cur));
#define PCH(PV)                                                                         \
    case PV:                                                                            \
        hipLaunchKernelGGL((k_pchol<PV>), dim3(1), dim3(64), 0, s, dG, pass,             \
                           dtol_abs * dtol_abs, dXm(), dBm(), dBacc(), pass == 0 ? 1 : 0, \
                           d_rank + slot);                                              \
        break;
            switch (P) {
                PCH(1) PCH(2) PCH(4) PCH(8) PCH(16)
                default:
                    set_error("block width %d is not a power of two <= 16", P);
                    return MCD_E_INVALID;
            }
#undef PCH
            T *out = pass == 0 ? W2 : dst;
            MCD_TRY(block_apply_dev(cur, 1, dXm(), out, false));
            cur = out;
        }
        MCD_HIP(hipMemcpyAsync(outB, dBacc(), PP() * sizeof(double), hipMemcpyDeviceToDevice, s));
        return MCD_OK;
    }

    // One block step j of the device form, up to W = the new residual block
    // (product, A_j, three-term update, reorthogonalisation).
    int step_dev(int j, int reorth) {
        MCD_TRY(apply_any(op, sizeof(T) == 8 ? MCD_F64 : MCD_F32, P, blk(j), W, s));
        MCD_TRY(gram_dev(blk(j), 1, W));
        // W -= Q_{j-1} B_j^T + Q_j A_j in one pass, block j at its offset from
        // block j - 1 (negative where the ring of three wraps), so a ring and
        // a full store give the same W bit for bit
        hipLaunchKernelGGL(k_sym_pair, dim3(1), dim3(64), 0, s, P, dG, dA(j),
                           j > 0 ? dB(j) : nullptr, dC2());
        MCD_HIP(hipGetLastError());
        if (j > 0)
            MCD_TRY(block_apply_dev(blk(j - 1), 2, dC2(), W, true, (int64_t)(blk(j) - blk(j - 1))));
        else
            MCD_TRY(block_apply_dev(blk(0), 1, dC2() + PP(), W, true));
        for (int pass = 0; pass < reorth; pass++) {
            MCD_TRY(gram_dev(blk(0), j + 1, W));
            MCD_TRY(block_apply_dev(blk(0), j + 1, dG, W, true));
        }
        return MCD_OK;
    }

    // Host copies of the ranks [0, upto] and of T (enqueued; the caller
    // synchronises the stream before reading them).
    int fetch_ranks(int upto) {
        rank.resize(mb + 2);
        MCD_HIP(hipMemcpyAsync(rank.data(), d_rank, (size_t)(upto + 1) * sizeof(int),
                               hipMemcpyDeviceToHost, s));
        return MCD_OK;
    }
    int fetch_T() {
        hT.resize(nT());
        MCD_HIP(hipMemcpyAsync(hT.data(), dT, nT() * sizeof(double), hipMemcpyDeviceToHost, s));
        return MCD_OK;
    }
    // T of the first mm blocks (and R0) from the host copy; MCD_E_NUMERIC if
    // an entry in use is not finite
    int make_T(int mm, BandResult &out) const {
        const int PP = P * P;
        out = BandResult();
        out.P = P;
        out.B.assign(1, std::vector<double>());
        out.R0.assign(hT.begin() + (size_t)(2 * mb + 1) * PP, hT.begin() + (size_t)(2 * mb + 2) * PP);
        out.krylov = rank[0] > 0 ? rank[0] : 0;
        for (int j = 0; j < mm; j++) {
            out.A.emplace_back(hT.begin() + (size_t)j * PP, hT.begin() + (size_t)(j + 1) * PP);
            if (j > 0) {
                const size_t o = (size_t)(mb + j) * PP;
                out.B.emplace_back(hT.begin() + o, hT.begin() + o + PP);
                out.krylov += std::max(rank[j], 0);
            }
        }
        out.m = mm;
        auto finite = [](const std::vector<double> &v) {
            for (double x : v)
                if (!std::isfinite(x)) return false;
            return true;
        };
        bool ok = finite(out.R0);
        for (int j = 0; j < mm && ok; j++) ok = finite(out.A[j]) && (j == 0 || finite(out.B[j]));
        MCD_REQUIRE(ok, MCD_E_NUMERIC,
                    "band Lanczos: non-finite block tridiagonal entry (NaN or Inf in psi0 or H)");
        return MCD_OK;
    }

    // Host-driven form with one single-vector product per block column (the
    // unbatched reference): Gram matrices on the host, Gram-eigen QR.
    int run(double dtol_abs, int reorth, BandResult &out) {
        const int PP = P * P;
        out = BandResult();
        out.P = P;
        out.B.assign(1, std::vector<double>());
        int rk = 0;
        std::vector<double> R0;
        MCD_TRY(qr(W, blk(0), dtol_abs * dtol_abs, R0, &rk));
        out.R0 = R0;
        out.krylov = rk;
        if (rk == 0) {
            out.m = 0;
            return MCD_OK;
        }
        std::vector<double> G, C;
        for (int j = 0; j < mb; j++) {
            if (per_column) {
                for (int k = 0; k < P; k++) {
                    hipLaunchKernelGGL((k_column<T>), dim3(gridn(n, 256)), dim3(256), 0, s, n, P,
                                       k, blk(j), colbuf, 0);
                    MCD_TRY(apply_any(op, sizeof(T) == 8 ? MCD_F64 : MCD_F32, 1, colbuf,
                                      colbuf + n, s));
                    hipLaunchKernelGGL((k_column<T>), dim3(gridn(n, 256)), dim3(256), 0, s, n, P,
                                       k, W, colbuf + n, 1);
                }
                MCD_HIP(hipGetLastError());
            } else {
                MCD_TRY(apply_any(op, sizeof(T) == 8 ? MCD_F64 : MCD_F32, P, blk(j), W, s));
            }
            MCD_TRY(gram(blk(j), 1, W, G));
            std::vector<double> Aj(PP);
            for (int a = 0; a < P; a++)        // symmetrise the projected block
                for (int b = 0; b < P; b++) Aj[a * P + b] = 0.5 * (G[a * P + b] + G[b * P + a]);
            out.A.push_back(Aj);
            // W -= Q_j A_j + Q_{j-1} B_j^T
            MCD_TRY(block_apply(blk(j), 1, Aj, W, true));
            if (j > 0) {
                std::vector<double> Bt(PP);
                for (int a = 0; a < P; a++)
                    for (int b = 0; b < P; b++) Bt[a * P + b] = out.B[j][b * P + a];
                MCD_TRY(block_apply(blk(j - 1), 1, Bt, W, true));
            }
            for (int pass = 0; pass < reorth; pass++) {
                MCD_TRY(gram(blk(0), j + 1, W, C));
                MCD_TRY(block_apply(blk(0), j + 1, C, W, true));
            }
            if (j + 1 == mb) break;
            std::vector<double> Bn;
            MCD_TRY(qr(W, blk(j + 1), dtol_abs * dtol_abs, Bn, &rk));
            out.B.push_back(Bn);
            if (rk == 0) break;
            out.krylov += rk;
            if ((j + 1) % 8 == 0 && g_tol > 0.0) {
                out.m = (int)out.A.size();
                if (g_converged(out)) break;
            }
        }
        out.m = (int)out.A.size();
        return MCD_OK;
    }
};

// ---------------------------------------------------------------------------
// Kernels over many runs at once (block widths P = 8 and 16, packed-CSR
// operators): every kernel of a block step is one launch for all active
// runs.  A workgroup finds its run by binary search over the runs' first
// units (SpMM tiles, padded Gram chunks, apply row tiles) in a descriptor
// table and does exactly the work the one-run kernel does for that unit, so
// each run's numbers are bit for bit those of its own launches.
struct MRun {
    int64_t n;
    const int64_t *rowptr;
    const uint32_t *colw;
    const double *diag;
    const DevModel *model;
    void *Qs, *W, *W2;
    double *part, *dG, *dT;
    int *rank;
    int64_t chunk_rows;
    int32_t nch, pad;
    int64_t tile0, chunk0, row0;
};

// which: 0 tiles, 1 chunks, 2 apply row tiles; the last run whose first unit
// is <= u (runs with no units are skipped over)
__device__ __forceinline__ int mr_find(const MRun *__restrict__ R, int nrun, int64_t u,
                                       int which) {
    int lo = 0, hi = nrun - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t f = which == 0 ? R[mid].tile0 : which == 1 ? R[mid].chunk0 : R[mid].row0;
        if (f <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// A run's block buffer: kind 0 = W, 1 = W2, 2 = stored block `slot`.
template <typename T>
__device__ __forceinline__ T *mr_buf(const MRun &r, int kind, int slot, int P) {
    if (kind == 0) return (T *)r.W;
    if (kind == 1) return (T *)r.W2;
    return (T *)r.Qs + (int64_t)slot * r.n * P;
}

template <typename T, int NV, int CH, int WMAX>
__global__ __launch_bounds__(256) void k_mr_spmm(const MRun *__restrict__ R, int nrun,
                                                 int64_t total, int rpt, int slot) {
    const int64_t per = (total + kNumXcd - 1) / kNumXcd;
    const int64_t t = (int64_t)(blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
    if (t >= total) return;   // whole workgroup, before any barrier
    const MRun &r = R[mr_find(R, nrun, t, 0)];
    const int64_t rbeg = (t - r.tile0) * rpt;
    block_csr_v_tile<T, NV, CH, WMAX>(r.rowptr, r.colw, r.model, r.diag, mr_buf<T>(r, 2, slot, NV),
                                      (T *)r.W, rbeg, min(rbeg + (int64_t)rpt, r.n));
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_mr_gram(const MRun *__restrict__ R, int nrun, int nm,
                                                 int qkind, int qslot, int xkind) {
    constexpr int MB = gram_blocks<T>();
    const int nmg = (nm + MB - 1) / MB;
    const int64_t u = blockIdx.x;
    const MRun &r = R[mr_find(R, nrun, u / nmg, 1)];
    const int64_t v = u - r.chunk0 * nmg;
    const int k = (int)(v / 8), mg = k % nmg, chunk = (k / nmg) * 8 + (int)(v % 8);
    if (chunk >= r.nch) return;   // whole workgroup, before any barrier
    const int m0 = mg * MB;
    gram_mfma_unit<T, P>(r.n, r.chunk_rows, r.nch, mr_buf<T>(r, qkind, qslot, P), r.n * P, m0,
                         min(MB, nm - m0), mr_buf<T>(r, xkind, 0, P), r.part, chunk);
}

__global__ __launch_bounds__(256) void k_mr_gram_reduce(const MRun *__restrict__ R, int nrun,
                                                        int nm, int PP) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int per = nm * PP;
    if (w >= (int64_t)nrun * per) return;   // whole wavefront
    const MRun &r = R[w / per];
    gram_reduce_wave(r.nch, PP, r.part, r.dG, (int)(w % per), threadIdx.x & 63);
}

__global__ __launch_bounds__(64) void k_mr_sym_pair(const MRun *__restrict__ R, int P, int mb,
                                                    int j) {
    const MRun &r = R[blockIdx.x];
    const int PP = P * P;
    sym_pair_body(P, r.dG, r.dT + (size_t)j * PP,
                  j > 0 ? r.dT + (size_t)(mb + j) * PP : nullptr, r.dT + (size_t)(2 * mb + 5) * PP);
}

// dst (-)= sum_{m < nm} src_m C_m: src = buffer qkind (stored blocks from
// qslot on, qstep slots apart: -2 where a ring of three wraps), C = the
// run's dT (ckind 0) or dG (1) at offset coff.
template <typename T, int P>
__global__ __launch_bounds__(BS) void k_mr_apply(const MRun *__restrict__ R, int nrun, int nm,
                                                 int qkind, int qslot, int qstep, int ckind,
                                                 int64_t coff, int dkind, int dslot, int sub) {
    const int64_t u = blockIdx.x;
    const MRun &r = R[mr_find(R, nrun, u, 2)];
    const double *__restrict__ C = (ckind == 0 ? r.dT : r.dG) + coff;
    const int64_t row = (u - r.row0) * BS + threadIdx.x;
    if (row < r.n)
        block_apply_row<T, P>(row, nm, mr_buf<T>(r, qkind, qslot, P), (int64_t)qstep * r.n * P, C,
                              mr_buf<T>(r, dkind, dslot, P), sub);
}

template <int P>
__global__ __launch_bounds__(64) void k_mr_pchol(const MRun *__restrict__ R, int mb, int mode,
                                                 double thr_abs, int init, int slot) {
    const MRun &r = R[blockIdx.x];
    constexpr int PP = P * P;
    double *Xm = r.dT + (size_t)(2 * mb + 2) * PP;
    pchol_body<P>(r.dG, mode, thr_abs, Xm, Xm + PP, Xm + 2 * PP, init, r.rank + slot);
}

// the QR factor (Bacc) of every run to its place in dT (offset dst_off)
__global__ __launch_bounds__(64) void k_mr_copy_factor(const MRun *__restrict__ R, int PP, int mb,
                                                       int64_t dst_off) {
    const MRun &r = R[blockIdx.x];
    const double *Bacc = r.dT + (size_t)(2 * mb + 4) * PP;
    for (int e = threadIdx.x; e < PP; e += 64) r.dT[dst_off + e] = Bacc[e];
}

// The descriptor table of the active runs (rebuilt, after a synchronisation,
// whenever the active set changes) and the fused step.
template <typename T>
struct MRTable {
    std::vector<MRun> host;
    MRun *dev = nullptr;       // workspace piece with room for every run
    int nrun = 0, P = 0, mb = 0, nstore = 0;
    int64_t tiles = 0, chunks = 0, rowt = 0;
    int rpt = 0, ch = 16;
    bool large = false;   // tiles with room for kBlockWordsLarge words
    hipStream_t s = nullptr;

    static bool usable(const std::vector<BandRun<T> *> &runs) {
        for (auto *r : runs)
            if (r->n > 0 && (r->op->storage != MCD_STORAGE_CSR || (r->P != 8 && r->P != 16)))
                return false;
        return true;
    }
    int slot(int j) const { return nstore == 3 ? j % 3 : j; }

    int build(const std::vector<BandRun<T> *> &act) {
        host.clear();
        tiles = chunks = rowt = 0;
        int64_t nnz = 0, rows = 0;
        constexpr int VN = 16 / sizeof(T);
        // one-pass tiles (block_tile) that fit every run's row blocks
        {
            const int L = act.empty() ? 1 : std::max(1, act[0]->P / VN);
            int rpb = 256, rpb_l = 256;
            for (auto *r : act) {
                rpb = std::min(rpb, r->op->rows_per_block);
                rpb_l = std::min(rpb_l, r->op->rows_per_block_l);
            }
            const BlockTile bt = block_tile(L, rpb, rpb_l);
            rpt = bt.rows;
            large = bt.large;
        }
        for (auto *r : act) {
            P = r->P;
            mb = r->mb;
            nstore = r->nstore;
            MRun d;
            memset(&d, 0, sizeof(d));
            d.n = r->n;
            d.rowptr = r->op->d_rowptr;
            d.colw = r->op->d_colw;
            d.diag = r->op->d_diag;
            d.model = r->op->d_model;
            d.Qs = r->Qs;
            d.W = r->W;
            d.W2 = r->W2;
            d.part = r->part;
            d.dG = r->dG;
            d.dT = r->dT;
            d.rank = r->d_rank;
            d.chunk_rows = r->chunk_rows;
            d.nch = r->nch;
            d.tile0 = tiles;
            d.chunk0 = chunks;
            d.row0 = rowt;
            tiles += (r->n + rpt - 1) / rpt;
            chunks += ((int64_t)r->nch + 7) / 8 * 8;
            rowt += (r->n + BS - 1) / BS;
            nnz += r->op->nnz;
            rows += r->n;
            host.push_back(d);
        }
        nrun = (int)host.size();
        ch = block_chunk(P / VN, (nnz < 4 * rows) ? 4 : (nnz < 10 * rows) ? 8 : 16);
        if (nrun > 0)
            MCD_HIP(hipMemcpyAsync(dev, host.data(), nrun * sizeof(MRun), hipMemcpyHostToDevice, s));
        return MCD_OK;
    }

    int spmm(int j) {
#define MRS(NV, CH, WM)                                                                      \
    hipLaunchKernelGGL((k_mr_spmm<T, NV, CH, WM>), dim3((unsigned)((tiles + 7) / 8 * 8)),    \
                       dim3(256), 0, s, dev, nrun, tiles, rpt, slot(j))
#define MRW(NV, CH) \
    do {                                                                                     \
        if (large) MRS(NV, CH, kBlockWordsLarge); else MRS(NV, CH, kStreamNnzMax);           \
    } while (0)
        if (P == 8) {
            if (ch == 4) MRW(8, 4); else if (ch == 8) MRW(8, 8); else MRW(8, 16);
        } else {
            if (ch == 4) MRW(16, 4); else if (ch == 8) MRW(16, 8); else MRW(16, 16);
        }
#undef MRW
#undef MRS
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    }
    int gram(int nm, int qkind, int qslot, int xkind) {
        const unsigned g = (unsigned)(chunks * ((nm + gram_blocks<T>() - 1) / gram_blocks<T>()));
        if (P == 8)
            hipLaunchKernelGGL((k_mr_gram<T, 8>), dim3(g), dim3(256), 0, s, dev, nrun, nm, qkind,
                               qslot, xkind);
        else
            hipLaunchKernelGGL((k_mr_gram<T, 16>), dim3(g), dim3(256), 0, s, dev, nrun, nm, qkind,
                               qslot, xkind);
        MCD_HIP(hipGetLastError());
        const int64_t waves = (int64_t)nrun * nm * P * P;
        hipLaunchKernelGGL(k_mr_gram_reduce, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s,
                           dev, nrun, nm, P * P);
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    }
    int apply(int nm, int qkind, int qslot, int ckind, int64_t coff, int dkind, int dslot,
              bool sub, int qstep = 1) {
        if (P == 8)
            hipLaunchKernelGGL((k_mr_apply<T, 8>), dim3((unsigned)rowt), dim3(BS), 0, s, dev, nrun,
                               nm, qkind, qslot, qstep, ckind, coff, dkind, dslot, sub ? 1 : 0);
        else
            hipLaunchKernelGGL((k_mr_apply<T, 16>), dim3((unsigned)rowt), dim3(BS), 0, s, dev, nrun,
                               nm, qkind, qslot, qstep, ckind, coff, dkind, dslot, sub ? 1 : 0);
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    }
    // QR of W into stored block `dslot`: two pivoted-Cholesky passes through
    // W2, the factor to dT[dst_off], the rank to rank[rslot]
    int qr(int dslot, int64_t dst_off, int rslot, double dtol_abs) {
        const int PP = P * P;
        const int64_t xm_off = (int64_t)(2 * mb + 2) * PP;
        for (int pass = 0; pass < 2; pass++) {
            MCD_TRY(gram(1, pass == 0 ? 0 : 1, 0, pass == 0 ? 0 : 1));
            if (P == 8)
                hipLaunchKernelGGL((k_mr_pchol<8>), dim3(nrun), dim3(64), 0, s, dev, mb, pass,
                                   dtol_abs * dtol_abs, pass == 0 ? 1 : 0, rslot);
            else
                hipLaunchKernelGGL((k_mr_pchol<16>), dim3(nrun), dim3(64), 0, s, dev, mb, pass,
                                   dtol_abs * dtol_abs, pass == 0 ? 1 : 0, rslot);
            MCD_HIP(hipGetLastError());
            MCD_TRY(apply(1, pass == 0 ? 0 : 1, 0, 0, xm_off, pass == 0 ? 1 : 2, dslot, false));
        }
        hipLaunchKernelGGL(k_mr_copy_factor, dim3(nrun), dim3(64), 0, s, dev, PP, mb, dst_off);
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    }
    // block step j up to the new residual block in W (as BandRun::step_dev)
    int step(int j, int reorth) {
        const int PP = P * P;
        MCD_TRY(spmm(j));
        MCD_TRY(gram(1, 2, slot(j), 0));
        hipLaunchKernelGGL(k_mr_sym_pair, dim3(nrun), dim3(64), 0, s, dev, P, mb, j);
        MCD_HIP(hipGetLastError());
        const int64_t c2 = (int64_t)(2 * mb + 5) * PP;
        if (j > 0)   // one pass, block j at its (signed) slot offset from block j - 1
            MCD_TRY(apply(2, 2, slot(j - 1), 0, c2, 0, 0, true, slot(j) - slot(j - 1)));
        else
            MCD_TRY(apply(1, 2, slot(0), 0, c2 + PP, 0, 0, true));
        const int group = std::max(1, (48 * 1024) / (PP * 8));
        for (int pass = 0; pass < reorth; pass++) {
            MCD_TRY(gram(j + 1, 2, 0, 0));
            for (int g0 = 0; g0 <= j; g0 += group)
                MCD_TRY(apply(std::min(group, j + 1 - g0), 2, g0, 1, (int64_t)g0 * PP, 0, 0, true));
        }
        return MCD_OK;
    }
};

// Block Lanczos of every run in `runs` (device form) in lockstep: at block
// step j every active run does its product, A_j, update,
// reorthogonalisation and QR, each kernel enqueued for all runs before the
// next, on one stream.  Every 8 steps the ranks (and, with g_tol, G at the
// check points) are read back with one synchronisation for all runs; a run
// whose Krylov space is exhausted or whose G has settled stops there.  Each
// run's arithmetic depends on that run alone, so its result is the same in
// any company.  Each run's start block is in its W.
template <typename T>
using BlockHook = std::function<int(BandRun<T> &, int)>;

// on_block (optional) is called for each run and block j once Q_j is formed
// (after its QR, before any later block overwrites a ring slot); it enqueues
// its work on the stream.
template <typename T>
static int run_lockstep(std::vector<BandRun<T> *> &runs, double dtol_abs, int reorth,
                        hipStream_t s, const BlockHook<T> *on_block = nullptr) {
    int mb = 0;
    std::vector<BandRun<T> *> act;
    for (auto *r : runs) {
        r->m = 0;
        r->active = r->n > 0;
        r->gprev.clear();
        mb = std::max(mb, r->mb);
        if (r->active) act.push_back(r);
    }
    // fused launches over all runs when every operator is a packed CSR and
    // P is 8 or 16; else each run's own launches
    MRTable<T> tab;
    tab.s = s;
    const bool fused = !act.empty() && MRTable<T>::usable(act);
    Alloc tal;
    if (fused) {
        tal = act[0]->al;
        const hipError_t e = dmalloc((void **)&tab.dev, act.size() * sizeof(MRun), tal);
        if (e != hipSuccess) {
            set_error("band runs: workspace too small for the run table");
            return hip_status(e);
        }
    }
    auto done = [&](int rc) {
        if (tab.dev) {
            (void)hipStreamSynchronize(s);
            (void)dfree(tab.dev, tal);
        }
        return rc;
    };
#define LTRY(expr)                     \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ < 0) return done(rc_); \
    } while (0)
    const int PP0 = act.empty() ? 0 : act[0]->PP();
    if (fused) {
        LTRY(tab.build(act));
        LTRY(tab.qr(tab.slot(0), (int64_t)(2 * mb + 1) * PP0, 0, dtol_abs));
    } else {
        for (auto *r : act) LTRY(r->qr_dev(r->W, r->blk(0), r->dR0(), 0, dtol_abs));
    }
    for (auto *r : act) LTRY(r->fetch_ranks(0));
    if (hipStreamSynchronize(s) != hipSuccess) return done(MCD_E_HIP);
    for (auto *r : runs)
        if (r->active && r->rank[0] <= 0) r->active = false;
    if (on_block)
        for (auto *r : runs)
            if (r->active) LTRY((*on_block)(*r, 0));
    // The checks every 8 block steps read each run's ranks (and, with g_tol,
    // T) back to the host.  Without a per-block hook or a replay limit the
    // read-back goes to a pinned host buffer, asynchronously, and the host
    // takes the check's decision only after the next block step and QR are
    // enqueued, so the GPU works on them meanwhile; a run that stops at the
    // check drops the extra step (its m goes back to the check's), so every
    // run ends where a synchronous check would have ended it, with the same T.
    bool spec = on_block == nullptr && !act.empty();
    for (auto *r : runs)
        if (r->limit > 0) spec = false;   // a replay's stop is checked synchronously
    char *pin = nullptr;
    hipEvent_t pev = nullptr;
    std::vector<size_t> off_rank(runs.size(), 0), off_T(runs.size(), 0);
    if (spec) {
        size_t bytes = 0;
        for (size_t i = 0; i < runs.size(); i++) {
            if (runs[i]->n == 0) continue;
            off_rank[i] = bytes;
            bytes += ((size_t)(runs[i]->mb + 2) * sizeof(int) + 7) / 8 * 8;
            off_T[i] = bytes;
            bytes += runs[i]->nT() * sizeof(double);
        }
        if (hipHostMalloc((void **)&pin, std::max<size_t>(bytes, 8), 0) != hipSuccess) {
            (void)hipGetLastError();
            pin = nullptr;
            spec = false;
        } else if (hipEventCreateWithFlags(&pev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            pev = nullptr;
            spec = false;
        }
    }
    auto release_pin = [&]() {
        if (pev || pin) (void)hipStreamSynchronize(s);
        if (pev) (void)hipEventDestroy(pev);
        if (pin) (void)hipHostFree(pin);
        pev = nullptr;
        pin = nullptr;
    };
#undef LTRY
#define LTRY(expr)                     \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ < 0) {                 \
            release_pin();             \
            return done(rc_);          \
        }                              \
    } while (0)
    auto index_of = [&](const BandRun<T> *r) {
        return (size_t)(std::find(runs.begin(), runs.end(), r) - runs.begin());
    };
    // The check at block c of the runs `lst` (host copies of their ranks
    // [0, c] and, with g_tol, of T): a run whose Krylov space is exhausted
    // ends at its first zero rank; a run whose G at the check points has
    // settled since its previous check ends at c.
    auto check = [&](int c, const std::vector<BandRun<T> *> &lst) -> int {
        for (auto *r : lst)
            for (int z = 1; z <= c; z++)
                if (r->rank[z] == 0) {   // exhausted: blocks from z on are zero
                    r->m = z;
                    r->active = false;
                    break;
                }
        std::vector<BandRun<T> *> chk;
        for (auto *r : lst)
            if (r->active && r->g_tol > 0.0) chk.push_back(r);
        if (chk.empty()) return MCD_OK;
        // T of every checked run, then G at every (run, check point) pair in
        // one parallel loop (one set of host threads per check, each pair
        // its own output)
        std::vector<int> rcs(chk.size(), MCD_OK);
        std::vector<BandResult> tmp(chk.size());
        for (size_t i = 0; i < chk.size(); i++) rcs[i] = chk[i]->make_T(c, tmp[i]);
        std::vector<std::vector<cplx>> gz(chk.size());
        std::vector<std::pair<int, int>> pairs;
        for (size_t i = 0; i < chk.size(); i++) {
            if (rcs[i] != MCD_OK || !chk[i]->g_wanted(tmp[i])) continue;
            const size_t pp = (size_t)chk[i]->p_sel * chk[i]->p_sel;
            gz[i].resize(chk[i]->zcheck.size() * pp);
            for (int f = 0; f < (int)chk[i]->zcheck.size(); f++) pairs.emplace_back((int)i, f);
        }
        parallel_for((int)pairs.size(), [&](int w) {
            const int i = pairs[w].first, f = pairs[w].second;
            const int ps = chk[i]->p_sel;
            block_cf(tmp[i], chk[i]->zcheck[f], ps, gz[i].data() + (size_t)f * ps * ps);
        });
        for (size_t i = 0; i < chk.size(); i++) {
            MCD_TRY(rcs[i]);
            if (!gz[i].empty() && chk[i]->g_settled(std::move(gz[i]))) {
                chk[i]->active = false;
                chk[i]->m = c;
            }
        }
        return MCD_OK;
    };
    int pend_c = 0;                        // block of the check in flight (0: none)
    std::vector<BandRun<T> *> pend;        // its runs
    auto finish_pending = [&]() -> int {
        if (pend_c == 0) return MCD_OK;
        const int c = pend_c;
        pend_c = 0;
        if (hipEventSynchronize(pev) != hipSuccess) return MCD_E_HIP;
        for (auto *r : pend) {
            const size_t i = index_of(r);
            r->rank.resize(r->mb + 2);
            memcpy(r->rank.data(), pin + off_rank[i], (size_t)(c + 1) * sizeof(int));
            if (r->g_tol > 0.0) {
                r->hT.resize(r->nT());
                memcpy(r->hT.data(), pin + off_T[i], r->nT() * sizeof(double));
            }
        }
        return check(c, pend);
    };
    size_t built = act.size();
    auto refresh = [&]() -> int {   // the active set, and the fused table for it
        act.clear();
        for (auto *r : runs)
            if (r->active) act.push_back(r);
        if (fused && !act.empty() && act.size() != built) {   // the set changed
            MCD_TRY(tab.build(act));
            built = act.size();
        }
        return MCD_OK;
    };
    for (int j = 0; j < mb; j++) {
        LTRY(refresh());
        if (act.empty()) break;
        if (fused)
            LTRY(tab.step(j, reorth));
        else
            for (auto *r : act) LTRY(r->step_dev(j, reorth));
        for (auto *r : act) r->m = j + 1;
        if (j + 1 == mb) break;
        // a replay stops at its limit (before the QR of the next block)
        for (auto *r : runs)
            if (r->active && r->limit > 0 && r->m >= r->limit) r->active = false;
        LTRY(refresh());
        if (act.empty()) break;
        if (fused)
            LTRY(tab.qr(tab.slot(j + 1), (int64_t)(mb + j + 1) * PP0, j + 1, dtol_abs));
        else
            for (auto *r : act)
                LTRY(r->qr_dev(r->W, r->blk(j + 1), r->dB(j + 1), j + 1, dtol_abs));
        if (on_block)
            for (auto *r : act) LTRY((*on_block)(*r, j + 1));
        // the check at block j (if one is in flight), decided while block
        // step j and the QR of block j + 1 run
        LTRY(finish_pending());
        if ((j + 1) % 8 == 0) {
            if (spec) {
                for (auto *r : act) {
                    const size_t i = index_of(r);
                    if (hipMemcpyAsync(pin + off_rank[i], r->d_rank,
                                       (size_t)(j + 2) * sizeof(int), hipMemcpyDeviceToHost,
                                       s) != hipSuccess ||
                        (r->g_tol > 0.0 &&
                         hipMemcpyAsync(pin + off_T[i], r->dT, r->nT() * sizeof(double),
                                        hipMemcpyDeviceToHost, s) != hipSuccess)) {
                        release_pin();
                        return done(MCD_E_HIP);
                    }
                }
                if (hipEventRecord(pev, s) != hipSuccess) {
                    release_pin();
                    return done(MCD_E_HIP);
                }
                pend = act;
                pend_c = j + 1;
            } else {
                for (auto *r : act) {
                    LTRY(r->fetch_ranks(j + 1));
                    if (r->g_tol > 0.0) LTRY(r->fetch_T());
                }
                if (hipStreamSynchronize(s) != hipSuccess) {
                    release_pin();
                    return done(MCD_E_HIP);
                }
                LTRY(check(j + 1, act));
            }
        }
    }
    LTRY(finish_pending());
    release_pin();
#undef LTRY
#define LTRY(expr)                     \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ < 0) return done(rc_); \
    } while (0)
    // final ranks and T of every run
    for (auto *r : runs)
        if (r->n > 0) {
            LTRY(r->fetch_ranks(std::max(r->m - 1, 0)));
            LTRY(r->fetch_T());
        }
    if (hipStreamSynchronize(s) != hipSuccess) return done(MCD_E_HIP);
    for (auto *r : runs) {
        r->active = false;
        if (r->n == 0) {
            r->br = BandResult();
            r->br.P = r->P;
            continue;
        }
        if (r->rank[0] <= 0) r->m = 0;
        for (int z = 1; z < r->m; z++)
            if (r->rank[z] == 0) {
                r->m = z;
                break;
            }
        LTRY(r->make_T(r->m, r->br));
    }
#undef LTRY
    return done(MCD_OK);
}

// F~+- of the kept states for the selection (images c+_mu x or c_mu x,
// radix sort, unique; Eq. excited_subspace) and the operator on it.  The
// image buffers are scratch; the operator's pieces stay in the workspace
// (run.op, released with the run).  n_x = 0: the sector is empty.
template <typename T>
static int prepare_sector(const mcd_model *model, const uint64_t *keys_t, int64_t nt,
                          const SelOps &sel, bool create, const mcd_band_cfg *cfg, mcd_ws *ws,
                          hipStream_t s, BandRun<T> &run) {
    const Alloc A{ws};
    uint64_t *img = nullptr, *srt = nullptr, *uniq = nullptr;
    int64_t *d_nu = nullptr;
    void *tmp = nullptr;
    auto free_images = [&]() {
        (void)hipStreamSynchronize(s);
        for (void *p : {tmp, (void *)d_nu, (void *)uniq, (void *)srt, (void *)img})
            if (p) (void)dfree(p, A);
        img = srt = uniq = nullptr;
        d_nu = nullptr;
        tmp = nullptr;
    };
#define CK(expr)                                                              \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess) {                                               \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
            free_images();                                                    \
            return hip_status(e_);                                            \
        }                                                                     \
    } while (0)
    run.al.ws = ws;
    run.s = s;
    run.n = 0;
    const int64_t ni = nt * sel.n;
    CK(dmalloc((void **)&img, std::max<int64_t>(ni, 1) * sizeof(uint64_t), A));
    CK(dmalloc((void **)&srt, std::max<int64_t>(ni, 1) * sizeof(uint64_t), A));
    CK(dmalloc((void **)&uniq, std::max<int64_t>(ni, 1) * sizeof(uint64_t), A));
    CK(dmalloc((void **)&d_nu, sizeof(int64_t), A));
    hipLaunchKernelGGL(k_images, dim3(gridn(nt, 256)), dim3(256), 0, s, nt, keys_t, sel,
                       create ? 1 : 0, img);
    CK(hipGetLastError());
    size_t b1 = 0, b2 = 0;
    CK(hipcub::DeviceRadixSort::SortKeys(nullptr, b1, img, srt, (int)ni, 0, 64, s));
    CK(hipcub::DeviceSelect::Unique(nullptr, b2, srt, uniq, d_nu, (int)ni, s));
    CK(dmalloc((void **)&tmp, std::max(b1, b2), A));
    size_t t1 = std::max(b1, b2), t2 = t1;
    CK(hipcub::DeviceRadixSort::SortKeys(tmp, t1, img, srt, (int)ni, 0, 64, s));
    CK(hipcub::DeviceSelect::Unique(tmp, t2, srt, uniq, d_nu, (int)ni, s));
    int64_t nu = 0;
    CK(hipMemcpyAsync(&nu, d_nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    uint64_t lastk = 0;
    if (nu > 0) {
        CK(hipMemcpyAsync(&lastk, uniq + nu - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        if (lastk == kEmpty) nu--;
    }
#undef CK
    if (nu > 0) {
        mcd_op *op = nullptr;
        const int rc = op_create(model, uniq, nu, cfg->storage, 0, cfg->per_column != 0, ws, s, &op);
        if (rc < 0) {
            free_images();
            return rc;
        }
        run.op = op;
        run.n = nu;
    }
    free_images();   // the operator holds its own copy of the keys
    return MCD_OK;
}

// Pieces of a prepared run (n > 0): Krylov store, work blocks, Gram
// partials, coefficient store.  `plan` replays the takes on host bookkeeping
// instead (for the workspace-size answer).
template <typename T>
static size_t run_piece_sizes(const BandRun<T> &r, size_t out[9]) {
    const size_t PPb = (size_t)r.P * r.P * sizeof(double);
    out[0] = (size_t)r.nstore * r.n * r.P * sizeof(T);                   // Qs
    out[1] = (size_t)r.n * r.P * sizeof(T);                              // W
    out[2] = r.per_column ? 0 : (size_t)r.n * r.P * sizeof(T);           // W2
    out[3] = r.per_column ? (size_t)2 * r.n * sizeof(T) : 0;             // colbuf
    out[4] = (size_t)r.part_cap * sizeof(double);                        // part
    out[5] = (size_t)(r.mb + 1) * PPb;                                   // dG
    out[6] = (size_t)(r.mb + 1) * PPb;                                   // dC
    out[7] = r.nT() * sizeof(double);                                    // dT
    out[8] = (size_t)(r.mb + 2) * sizeof(int);                           // d_rank
    return 9;
}

template <typename T>
static void run_configure(BandRun<T> &r, const mcd_band_cfg *cfg, int P, bool store_all,
                          const SelOps &sel, const std::vector<cplx> *zcheck) {
    const int reorth = std::max(0, std::min(2, (int)cfg->reorth));
    r.P = P;
    r.mb = cfg->max_blocks;
    r.nstore = (reorth > 0 || store_all) ? cfg->max_blocks + 1 : 3;
    r.per_column = cfg->per_column != 0;
    r.g_tol = cfg->g_tol;
    r.p_sel = sel.n;
    if (zcheck) r.zcheck = *zcheck;
    r.set_chunks();
    r.part_cap = r.partials_needed();
}

template <typename T>
static int run_allocate(BandRun<T> &r) {
    size_t sz[9];
    run_piece_sizes(r, sz);
    void **dst[9] = {(void **)&r.Qs, (void **)&r.W, (void **)&r.W2, (void **)&r.colbuf,
                     (void **)&r.part, (void **)&r.dG, (void **)&r.dC, (void **)&r.dT,
                     (void **)&r.d_rank};
    for (int i = 0; i < 9; i++) {
        if (sz[i] == 0) continue;
        const hipError_t e = r.take(dst[i], sz[i]);
        if (e != hipSuccess) {
            set_error("band run: workspace too small for its blocks (%.1f MB more)",
                      sz[i] / 1048576.0);
            return hip_status(e);
        }
        if (i < 8) MCD_HIP(poison_fp(*dst[i], sz[i], r.al, r.s));   // all but d_rank
    }
    return MCD_OK;
}

// Start block c+_mu|psi> (c_mu|psi>) of the kept states scattered into W.
template <typename T>
static int run_start_block(BandRun<T> &r, const uint64_t *keys_t, const double *psi_t, int64_t nt,
                           const SelOps &sel, bool create) {
    MCD_HIP(hipMemsetAsync(r.W, 0, (size_t)r.n * r.P * sizeof(T), r.s));
    hipLaunchKernelGGL((k_start_block<T>), dim3(gridn(nt, 256)), dim3(256), 0, r.s, nt, keys_t,
                       psi_t, sel, create ? 1 : 0, r.op->d_hash, r.op->hash_mask, r.P, r.W);
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}

// Workspace extent after taking the pieces of `runs` (n > 0, not yet
// allocated), replayed on a copy of the workspace's bookkeeping.
template <typename T>
static size_t plan_runs(mcd_ws *ws, const std::vector<BandRun<T> *> &runs) {
    WsAlloc sim(0);
    {
        std::lock_guard<std::mutex> lock(ws->mu);
        sim = ws->a;
    }
    sim.grow_to(size_t(1) << 62);   // the same live pieces, an unbounded range
    size_t live = 0;
    for (auto *r : runs) {
        if (r->n == 0) continue;
        size_t sz[9];
        run_piece_sizes(*r, sz);
        for (int i = 0; i < 9; i++)
            if (sz[i]) (void)sim.alloc(sz[i]);
        live++;
    }
    if (live) (void)sim.alloc(live * sizeof(MRun));   // run_lockstep's table
    return sim.extent();
}

// Points where the convergence of G is checked: every frequency if there are
// at most 8, else the one closest to the real axis (smallest |w|) and 7 more
// evenly spaced; z = E0 + zeta (particle run) or E0 - zeta (hole run).
static void check_points(const mcd_band_cfg *cfg, int n_freq, const double *omega, double e0,
                         std::vector<cplx> &zp, std::vector<cplx> &zm) {
    std::vector<int> idx;
    if (n_freq <= 8) {
        for (int f = 0; f < n_freq; f++) idx.push_back(f);
    } else {
        int fmin = 0;
        for (int f = 1; f < n_freq; f++)
            if (fabs(omega[f]) < fabs(omega[fmin])) fmin = f;
        idx.push_back(fmin);
        for (int k = 0; k < 7; k++) idx.push_back((int)((int64_t)k * (n_freq - 1) / 6));
        std::sort(idx.begin(), idx.end());
        idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
    }
    zp.clear();
    zm.clear();
    for (int f : idx) {
        zp.push_back(e0 + freq_arg(cfg, omega[f]));
        zm.push_back(e0 - freq_arg(cfg, omega[f]));
    }
}

// The w_t cut of one ground state (Sec. Further truncation): the kept keys
// and the renormalised kept amplitudes (keys_t, psi_t: pieces of the
// workspace, released by the caller).
static int wt_cut(const uint64_t *keys_dev, int64_t n, const double *psi0_dev, double w_t,
                  mcd_ws *ws, hipStream_t s, uint64_t **keys_t_out, double **psi_t_out,
                  int64_t *n_keep_out) {
    const Alloc A{ws};
    double *w = nullptr, *w2 = nullptr, *scr = nullptr, *psi_t = nullptr;
    uint32_t *idx = nullptr, *idx2 = nullptr, *kept = nullptr;
    uint64_t *keys_t = nullptr;
    void *tmp = nullptr;
    *keys_t_out = nullptr;
    *psi_t_out = nullptr;
    auto scratch_free = [&]() {
        (void)hipStreamSynchronize(s);
        for (void *p : {tmp, (void *)scr, (void *)kept, (void *)idx2, (void *)idx, (void *)w2,
                        (void *)w})
            if (p) (void)dfree(p, A);
        tmp = scr = nullptr;
        kept = idx2 = idx = nullptr;
        w2 = w = nullptr;
    };
#define CK(expr)                                                              \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess) {                                               \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));         \
            scratch_free();                                                   \
            (void)dfree(psi_t, A);                                            \
            (void)dfree(keys_t, A);                                           \
            return hip_status(e_);                                            \
        }                                                                     \
    } while (0)
    MCD_REQUIRE(n < (int64_t(1) << 31), MCD_E_CAPACITY, "basis too large for the w_t sort");
    // kept outputs first (they outlive the scratch)
    CK(dmalloc((void **)&keys_t, n * sizeof(uint64_t), A));
    CK(dmalloc((void **)&psi_t, n * sizeof(double), A));
    CK(dmalloc((void **)&w, n * sizeof(double), A));
    CK(dmalloc((void **)&idx, n * sizeof(uint32_t), A));
    CK(dmalloc((void **)&kept, n * sizeof(uint32_t), A));
    CK(dmalloc((void **)&scr, (4096 + 8) * sizeof(double), A));
    CK(poison_fp(psi_t, n * sizeof(double), A, s));
    CK(poison_fp(w, n * sizeof(double), A, s));
    CK(poison_fp(scr, (4096 + 8) * sizeof(double), A, s));
    hipLaunchKernelGGL(k_weights, dim3(gridn(n, 256)), dim3(256), 0, s, n, psi0_dev, w, idx);
    CK(hipGetLastError());
    int64_t n_keep = n;
    if (w_t < 1.0) {
        CK(dmalloc((void **)&w2, n * sizeof(double), A));
        CK(dmalloc((void **)&idx2, n * sizeof(uint32_t), A));
        CK(poison_fp(w2, n * sizeof(double), A, s));
        size_t b1 = 0;
        CK(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, b1, w, w2, idx, idx2, (int)n, 0,
                                                        64, s));
        size_t b2 = 0;
        CK(hipcub::DeviceRadixSort::SortKeys(nullptr, b2, idx2, kept, (int)n, 0, 32, s));
        CK(dmalloc((void **)&tmp, std::max(b1, b2), A));
        size_t t1 = std::max(b1, b2);
        CK(hipcub::DeviceRadixSort::SortPairsDescending(tmp, t1, w, w2, idx, idx2, (int)n, 0, 64,
                                                        s));
        std::vector<double> hw(n);
        CK(hipMemcpyAsync(hw.data(), w2, n * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        double total = 0.0;
        for (int64_t i = 0; i < n; i++) total += hw[i];
        if (!std::isfinite(total) || !(total > 0.0)) {
            scratch_free();
            (void)dfree(psi_t, A);
            (void)dfree(keys_t, A);
            set_error("w_t cut: psi0 has no finite, nonzero weight");
            return MCD_E_NUMERIC;
        }
        double cum = 0.0;
        n_keep = n;
        for (int64_t i = 0; i < n; i++) {
            cum += hw[i] / total;
            if (cum >= w_t) {
                n_keep = i + 1;
                break;
            }
        }
        size_t t2 = std::max(b1, b2);
        CK(hipcub::DeviceRadixSort::SortKeys(tmp, t2, idx2, kept, (int)n_keep, 0, 32, s));
    } else {
        CK(hipMemcpyAsync(kept, idx, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_gather_kept, dim3(gridn(n_keep, 256)), dim3(256), 0, s, n_keep, kept,
                       keys_dev, psi0_dev, keys_t, psi_t);
    const unsigned nbn = std::min<unsigned>(gridn(n_keep, BS), 2048);
    hipLaunchKernelGGL(k_norm2, dim3(nbn), dim3(BS), 0, s, n_keep, psi_t, scr);
    hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nbn, scr, scr + 4096);
    hipLaunchKernelGGL(k_scale_by, dim3(gridn(n_keep, 256)), dim3(256), 0, s, n_keep, psi_t,
                       scr + 4096);
    CK(hipGetLastError());
    double nrm2 = 0.0;
    CK(hipMemcpyAsync(&nrm2, scr + 4096, sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
#undef CK
    scratch_free();
    if (!std::isfinite(nrm2) || !(nrm2 > 0.0)) {
        (void)dfree(psi_t, A);
        (void)dfree(keys_t, A);
        set_error("w_t cut: the kept ground state has norm^2 %g (NaN, Inf or zero in psi0)", nrm2);
        return MCD_E_NUMERIC;
    }
    *keys_t_out = keys_t;
    *psi_t_out = psi_t;
    *n_keep_out = n_keep;
    return MCD_OK;
}

// One instance of a (batched) Green-function call: its cut ground state and
// its two sector runs.
template <typename T>
struct Instance {
    const mcd_model *model = nullptr;
    const uint64_t *keys = nullptr;
    int64_t n = 0;
    const double *psi = nullptr;
    double e0 = 0.0;
    double *G_out = nullptr, *Gp_out = nullptr, *Gm_out = nullptr;
    uint64_t *keys_t = nullptr;   // kept states and amplitudes (workspace)
    double *psi_t = nullptr;
    int64_t n_keep = 0;
    BandRun<T> plus, minus;
};

// G of one instance from its two runs (resolvents at every frequency, one
// host thread per frequency).
template <typename T>
static void assemble_green(const Instance<T> &in, int p, int n_freq, const double *omega,
                           const mcd_band_cfg *cfg) {
    const BandResult &brp = in.plus.br, &brm = in.minus.br;
    const double e0 = in.e0;
    parallel_for(n_freq, [&](int f) {
        std::vector<cplx> g(p * p);
        cplx *Gf = (cplx *)in.G_out + (size_t)f * p * p;
        for (int e = 0; e < p * p; e++) Gf[e] = 0.0;
        if (brp.m > 0) {
            block_cf(brp, e0 + freq_arg(cfg, omega[f]), p, g.data());
            for (int e = 0; e < p * p; e++) {
                Gf[e] += g[e];
                if (in.Gp_out) ((cplx *)in.Gp_out)[(size_t)f * p * p + e] = g[e];
            }
        } else if (in.Gp_out) {
            for (int e = 0; e < p * p; e++) ((cplx *)in.Gp_out)[(size_t)f * p * p + e] = 0.0;
        }
        if (brm.m > 0) {
            block_cf(brm, e0 - freq_arg(cfg, omega[f]), p, g.data());
            for (int e = 0; e < p * p; e++) {
                Gf[e] -= g[e];
                if (in.Gm_out) ((cplx *)in.Gm_out)[(size_t)f * p * p + e] = -g[e];
            }
        } else if (in.Gm_out) {
            for (int e = 0; e < p * p; e++) ((cplx *)in.Gm_out)[(size_t)f * p * p + e] = 0.0;
        }
    });
}


// Green functions of instances [0, K): cut, F~+- and operators for a group
// of instances at a time (as many as the workspace holds: their runs are
// planned on the host before any block is taken), then all runs of the group
// in lockstep.  plan_need != nullptr: prepare the first instance only and
// report the bytes it needs (no block steps; MCD_E_WORKSPACE when even the
// preparation did not fit, with the workspace's `need` as a lower bound).
// keep_runs (one instance): its runs stay (operators, Krylov blocks, T) for
// the caller to release.
template <typename T>
static int band_green_multi(std::vector<Instance<T> *> &inst, const SelOps &sel, int n_freq,
                            const double *omega, const mcd_band_cfg *cfg, mcd_ws *ws,
                            hipStream_t s, bool store_all, size_t *plan_need, bool keep_runs,
                            mcd_solve_info *info) {
    const double t0 = wall_ms();
    const int K = (int)inst.size();
    int P = 1;
    while (P < sel.n) P <<= 1;
    const int p = sel.n;
    const int reorth = std::max(0, std::min(2, (int)cfg->reorth));
    const double dtol_abs = cfg->dtol;
    const Alloc A{ws};
    auto drop_inst = [&](Instance<T> &in) {
        (void)hipStreamSynchronize(s);
        in.plus.release();
        in.minus.release();
        (void)dfree(in.psi_t, A);
        (void)dfree(in.keys_t, A);
        in.psi_t = nullptr;
        in.keys_t = nullptr;
    };
    mcd_solve_info agg;
    memset(&agg, 0, sizeof(agg));
    size_t need_max = 0;
    {   // the size answers below measure this call alone
        std::lock_guard<std::mutex> lock(ws->mu);
        ws->a.restart_extent();
    }
    int k0 = 0;
    while (k0 < K) {
        // prepare instances k0, k0 + 1, ... while their runs fit
        int k1 = k0;
        std::vector<BandRun<T> *> group;
        for (; k1 < K; k1++) {
            Instance<T> &in = *inst[k1];
            std::vector<cplx> zp, zm;
            check_points(cfg, n_freq, omega, in.e0, zp, zm);
            int rc = wt_cut(in.keys, in.n, in.psi, cfg->w_t, ws, s, &in.keys_t, &in.psi_t,
                            &in.n_keep);
            if (rc >= 0) rc = prepare_sector<T>(in.model, in.keys_t, in.n_keep, sel, true, cfg, ws, s, in.plus);
            if (rc >= 0) rc = prepare_sector<T>(in.model, in.keys_t, in.n_keep, sel, false, cfg, ws, s, in.minus);
            if (rc >= 0) {
                run_configure(in.plus, cfg, P, store_all, sel, &zp);
                run_configure(in.minus, cfg, P, store_all, sel, &zm);
            }
            size_t need = 0;
            if (rc >= 0) {
                std::vector<BandRun<T> *> g2 = group;
                g2.push_back(&in.plus);
                g2.push_back(&in.minus);
                need = plan_runs<T>(ws, g2);
            }
            const bool fits = rc >= 0 && need <= ws->a.size();
            if (rc >= 0 && fits) {
                group.push_back(&in.plus);
                group.push_back(&in.minus);
                need_max = std::max(need_max, need);
                if (plan_need) {   // the size answer: this instance, as the call would take it
                    k1++;
                    break;
                }
                continue;
            }
            // does not fit (or failed): undo this instance
            const int rc_keep = rc;
            drop_inst(in);
            if (rc_keep < 0 && rc_keep != MCD_E_WORKSPACE) {
                for (int k = k0; k < k1; k++) drop_inst(*inst[k]);
                return rc_keep;
            }
            if (plan_need) {
                if (rc_keep >= 0) {
                    *plan_need = std::max(need_max, need);
                    return MCD_OK;
                }
                size_t nd = 0;
                {
                    std::lock_guard<std::mutex> lock(ws->mu);
                    nd = ws->a.need();
                }
                *plan_need = std::max(need_max, nd);
                set_error("band workspace size: the probe workspace is too small for the "
                          "preparation (grow it to %zu bytes)", *plan_need);
                return MCD_E_WORKSPACE;
            }
            if (k1 == k0) {   // not even one instance fits
                std::lock_guard<std::mutex> lock(ws->mu);
                if (rc_keep >= 0) ws->a.set_need(need);
                set_error("band Green function: the workspace (%zu bytes) holds no instance "
                          "(instance %d needs %zu bytes)", ws->a.size(), k1,
                          rc_keep >= 0 ? need : ws->a.need());
                return MCD_E_WORKSPACE;
            }
            break;
        }
        if (plan_need) {
            for (int k = k0; k < k1; k++) drop_inst(*inst[k]);
            *plan_need = need_max;
            return MCD_OK;
        }
        // blocks of the group's runs, start blocks; the cut states go back
        int rc = MCD_OK;
        for (int k = k0; k < k1 && rc >= 0; k++) {
            Instance<T> &in = *inst[k];
            for (int side = 0; side < 2 && rc >= 0; side++) {
                BandRun<T> &r = side == 0 ? in.plus : in.minus;
                if (r.n == 0) continue;
                rc = run_allocate(r);
                if (rc >= 0) rc = run_start_block(r, in.keys_t, in.psi_t, in.n_keep, sel, side == 0);
            }
        }
        if (rc >= 0) rc = hipStreamSynchronize(s) == hipSuccess ? MCD_OK : MCD_E_HIP;
        for (int k = k0; k < k1; k++) {
            (void)dfree(inst[k]->psi_t, A);
            (void)dfree(inst[k]->keys_t, A);
            inst[k]->psi_t = nullptr;
            inst[k]->keys_t = nullptr;
        }
        if (rc >= 0) {
            if (cfg->per_column) {
                for (auto *r : group) {
                    if (r->n == 0) {
                        r->br = BandResult();
                        r->br.P = P;
                        continue;
                    }
                    rc = r->run(dtol_abs, reorth, r->br);
                    if (rc < 0) break;
                }
            } else {
                rc = run_lockstep<T>(group, dtol_abs, reorth, s);
            }
        }
        if (rc < 0) {
            for (int k = k0; k < k1; k++) drop_inst(*inst[k]);
            return rc;
        }
        for (int k = k0; k < k1; k++) {
            Instance<T> &in = *inst[k];
            if (in.G_out) assemble_green(in, p, n_freq, omega, cfg);
            agg.iters = std::max(agg.iters, std::max(in.plus.br.m, in.minus.br.m));
            agg.krylov_dim += in.plus.br.krylov + in.minus.br.krylov;
            agg.n_plus += in.plus.n;
            agg.n_minus += in.minus.n;
            agg.n_truncated += in.n_keep;
        }
        if (!keep_runs)
            for (int k = k0; k < k1; k++) drop_inst(*inst[k]);
        k0 = k1;
    }
    if (plan_need) *plan_need = need_max;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = agg.iters;
        info->converged = 1;
        info->e0 = K == 1 ? inst[0]->e0 : 0.0;
        info->solve_ms = wall_ms() - t0;
        info->krylov_dim = agg.krylov_dim;
        info->n_plus = agg.n_plus;
        info->n_minus = agg.n_minus;
        info->n_truncated = agg.n_truncated;
    }
    return MCD_OK;
}

// ---------------------------------------------------------------------------
// Reverse-mode derivative of G (vector-Jacobian product).

// lam[r] += sum_q sign * W[row(c_q x_r)][q]: the transpose of k_start_block
// (adjoint of the start block with respect to psi0).
template <typename T>
__global__ void k_start_block_t(int64_t m, const uint64_t *__restrict__ keys, SelOps sel,
                                int create, const HashSlot *__restrict__ h, uint64_t hmask, int P,
                                const T *__restrict__ W, double *__restrict__ lam) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const uint64_t k = keys[r];
    const uint32_t up = (uint32_t)(k >> 32), dn = (uint32_t)k;
    double acc = 0.0;
    for (int q = 0; q < sel.n; q++) {
        uint64_t t;
        if (!image(k, sel.orb[q], sel.spin[q], create != 0, &t)) continue;
        const int64_t row = hash_find(h, hmask, t);
        if (row >= 0) acc += jw_sign(up, dn, sel.orb[q], sel.spin[q]) * (double)W[row * P + q];
    }
    lam[r] += acc;
}

// The adjoint's weight matrix in symmetric form, for a store holding every
// Krylov block: Mp[i][j] = sg (A[i].B[j] + A[j].B[i]) = (M + M^T)[i][j] with
// M = sg A B^T (A, B: KP x K2 row-major float64), Mp [S][S] row-major in the
// store's type, zero past KP.  16 x 16 tiles, the four row panels staged
// through LDS in steps of 32 of k, one accumulator per dot summed in k order.
template <typename T>
__global__ __launch_bounds__(256) void k_sym_gram(int KP, int K2, int S, double sg,
                                                 const double *__restrict__ A,
                                                 const double *__restrict__ B,
                                                 T *__restrict__ Mp) {
    constexpr int TW = 16, KC = 32;
    __shared__ double Ai[TW][KC + 1], Bj[TW][KC + 1], Aj[TW][KC + 1], Bi[TW][KC + 1];
    const int tx = threadIdx.x, ty = threadIdx.y, t = ty * TW + tx;
    const int i0 = blockIdx.y * TW, j0 = blockIdx.x * TW;
    double s1 = 0.0, s2 = 0.0;
    for (int k0 = 0; k0 < K2; k0 += KC) {
        for (int e = t; e < TW * KC; e += TW * TW) {
            const int rr = e / KC, kk = e % KC, k = k0 + kk;
            const int ri = i0 + rr, rj = j0 + rr;
            const bool kin = k < K2;
            Ai[rr][kk] = kin && ri < KP ? A[(size_t)ri * K2 + k] : 0.0;
            Bi[rr][kk] = kin && ri < KP ? B[(size_t)ri * K2 + k] : 0.0;
            Aj[rr][kk] = kin && rj < KP ? A[(size_t)rj * K2 + k] : 0.0;
            Bj[rr][kk] = kin && rj < KP ? B[(size_t)rj * K2 + k] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KC; kk++) {
            s1 = fma(Ai[ty][kk], Bj[tx][kk], s1);
            s2 = fma(Aj[tx][kk], Bi[ty][kk], s2);
        }
        __syncthreads();
    }
    const int i = i0 + ty, j = j0 + tx;
    if (i < S && j < S) Mp[(size_t)i * S + j] = (T)(sg * s1 + sg * s2);
}

// Zt += Q M for the adjoint: Q consecutive Krylov blocks (n x P each, P a
// power of two; Q[r][k] = block k / P, row r, column k % P, k < KP), M
// row-major with S columns and Zt [n][S] row-major, S a multiple of 128.  A
// workgroup of four wavefronts makes one 128 x 128 tile of Zt, each wavefront
// a 64 x 64 quarter as 4 x 4 MFMA 16x16x4 products (float32 or float64 in,
// same type accumulated), with both operands staged through LDS in steps of
// 128 bytes of k.  Tiles are handed out XCD-major, so the S / 128 column tiles
// of one row tile run on one XCD and share its L2 copy of the Q rows.  M is
// read for rows < KP rounded up to 8 x 16 bytes of k (finite there; the
// products with rows past KP meet zero Q values).  Each element of Zt gets
// its product over the KP terms, rounded, added once.
template <typename T>
__global__ __launch_bounds__(256) void k_rows_times(int64_t n, int S, int KP, int pl,
                                                   const T *__restrict__ Q,
                                                   const T *__restrict__ M, T *__restrict__ Zt) {
    constexpr int BM = 128, BN = 128, U = 16 / sizeof(T), BK = 8 * U;
    constexpr int LA = BK + U, LB = BN + 4 * U;   // padded LDS rows (conflict-free reads)
    using V16 = T __attribute__((ext_vector_type(16 / sizeof(T))));
    using V4 = T __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) T As[BM * LA];   // As[row][k]
    __shared__ __attribute__((aligned(16))) T Bs[BK * LB];   // Bs[k][col]
    const int P = 1 << pl;
    const int ntc = S / BN;
    const int64_t ntr = (n + BM - 1) / BM, G = ntr * ntc, Gp = (G + 7) / 8 * 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * (Gp / 8) + blockIdx.x / 8;
    if (t >= G) return;   // whole workgroup, before any barrier
    const int64_t r0 = (t / ntc) * BM;
    const int c0 = (int)(t % ntc) * BN;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = (wid >> 1) * 64, wc = (wid & 1) * 64;
    const int li = lane & 15, lk = lane >> 4;
    V4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = (V4)(T)0;
    const int kend = (KP + BK - 1) / BK * BK;   // Q is zero past KP
    for (int k0 = 0; k0 < kend; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; q++) {   // A: 128 rows x 8 units of 16 bytes
            const int e = tid + q * 256, row = e >> 3, ku = (e & 7) * U, kg = k0 + ku;
            const int64_t r = r0 + row;
            V16 v = (V16)(T)0;
            if (r < n && kg < KP) {
                if (P >= U) {   // the unit lies in one block
                    v = *(const V16 *)(Q + ((((int64_t)(kg >> pl) * n + r) << pl) | (kg & (P - 1))));
                } else {
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const int k = kg + u;
                        if (k < KP) v[u] = Q[(((int64_t)(k >> pl) * n + r) << pl) | (k & (P - 1))];
                    }
                }
            }
            *(V16 *)(As + row * LA + ku) = v;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {   // B: BK rows x (BN / U) units
            const int e = tid + q * 256, kr = e / (BN / U), cu = (e % (BN / U)) * U;
            *(V16 *)(Bs + kr * LB + cu) = *(const V16 *)(M + (int64_t)(k0 + kr) * S + c0 + cu);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; i++) a[i] = As[(wr + i * 16 + li) * LA + kk + lk];
#pragma unroll
            for (int j = 0; j < 4; j++) b[j] = Bs[(kk + lk) * LB + wc + j * 16 + li];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if constexpr (sizeof(T) == 4)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // value v of a lane is D[4 (lane / 16) + v][lane % 16] of its 16 x 16 product
    // for float32 and D[lane / 16 + 4 v][lane % 16] for float64
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int64_t r = r0 + wr + i * 16 + (sizeof(T) == 4 ? 4 * lk + v : lk + 4 * v);
            if (r >= n) continue;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                T *z = Zt + r * S + c0 + wc + j * 16 + li;
                *z = *z + acc[i][j][v];
            }
        }
}

static constexpr int kCWaves = 4;
static constexpr int kMaxParams = MCD_MAX_BONDS + 2 * MCD_MAX_ORB;

// part[p * gridDim.x + block] = sum over this workgroup's rows r of
//   sum_a L[r][a] (dH/dtheta_p R)[r][a]
// for the merged bonds p < nb, then U_i (p = nb + i) and eps_i (nb + no + i):
// over all rows, tr(L^T dH_p R).  L and R are row-major [n][S] (columns
// a < KP used; R zero past KP).  One wavefront per row r.  The lanes look up
// all of the row's hop targets at once (lane 2q + s: bond q, spin s), the
// row L[r] is loaded once into registers (NR
// values per lane; NR = 0 re-reads it, any S), and the hops are then taken in
// lane order (bond by bond, up spin first), each a gather of the contiguous
// row Rt[col] with all NR loads issued together: loads past column S read the
// next row (or a zeroed tail of at least 64 (NR - S / 64) values after the
// last row) and meet zero weights.  Each wave keeps its own accumulators
// (fixed order).  SYM: L is instead a block-major Krylov store (column a =
// block a >> pl, entry a & (2^pl - 1)) and Rt = L (M + M^T) for the weight M:
// a hop pair r <-> c (same bond, same sign both ways) contributes
// L[r].(L M)[c] + L[c].(L M)[r] = L[r].Rt[c], so only hops with c > r are
// taken (half the gathers) and the diagonal term is L[r].Rt[r] / 2; the sums
// are then those of tr(L^T dH_p L M).
template <typename T, int NR, bool SYM>
__global__ __launch_bounds__(64 * kCWaves) void k_contract_rows(
    int64_t n, const uint64_t *__restrict__ keys, const DevModel *__restrict__ m,
    const HashSlot *__restrict__ h, uint64_t hmask, const T *__restrict__ L, int KP, int pl,
    const T *__restrict__ Rt, int S, double *__restrict__ part) {
    __shared__ double acc[kCWaves][kMaxParams];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nb = m->n_bonds, no = m->n_orb, np = nb + 2 * no;
    for (int i = lane; i < np; i += 64) acc[wid][i] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kCWaves + wid; r < n;
         r += (int64_t)gridDim.x * kCWaves) {
        const uint64_t key = keys[r];
        const uint32_t up = (uint32_t)(key >> 32), dn = (uint32_t)key;
        auto lval = [&](int a) -> T {
            if (a >= KP) return (T)0;
            if constexpr (SYM)   // block-major Krylov store
                return L[(((int64_t)(a >> pl) * n + r) << pl) | (a & ((1 << pl) - 1))];
            return L[r * (int64_t)S + a];
        };
        T qv[NR > 0 ? NR : 1];
        if constexpr (NR > 0) {
#pragma unroll
            for (int i = 0; i < NR; i++) qv[i] = lval(lane + 64 * i);
        }
        // sum_a L[r][a] Rt[col][a] over the wave (result in every lane)
        auto rowdot = [&](int64_t col) {
            const T *__restrict__ rc = Rt + col * (int64_t)S;
            double sum = 0.0;
            if constexpr (NR > 0) {
                T rv[NR];
#pragma unroll
                for (int i = 0; i < NR; i++) rv[i] = rc[lane + 64 * i];
#pragma unroll
                for (int i = 0; i < NR; i++) sum += (double)qv[i] * (double)rv[i];
            } else {
                for (int a = lane; a < S; a += 64) sum += (double)lval(a) * (double)rc[a];
            }
            return wave_sum(sum);
        };
        for (int base = 0; base < 2 * nb; base += 64) {
            const int hl = base + lane;
            int64_t col = -1;
            int neg = 0;
            if (hl < 2 * nb) {
                const uint32_t mask = m->bonds[hl >> 1].mask, between = m->bonds[hl >> 1].between;
                const uint32_t sp = (hl & 1) ? dn : up;
                if (__popc(sp & mask) == 1) {
                    col = hash_find(h, hmask, key ^ ((uint64_t)mask << ((hl & 1) ? 0 : 32)));
                    neg = __popc(sp & between) & 1;
                    if (SYM && col <= r) col = -1;   // each pair once (from its lower row)
                }
            }
            uint64_t live = __ballot(col >= 0);
            int cur = -1;
            double c = 0.0;
            while (live) {
                const int l = __ffsll((unsigned long long)live) - 1;
                live &= live - 1;
                // the hop of lane l, read into scalar registers (uniform)
                const uint32_t clo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)col, l);
                const uint32_t chi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(col >> 32), l);
                const int64_t cl = (int64_t)(((uint64_t)chi << 32) | clo);
                const int ng = __builtin_amdgcn_readlane(neg, l);
                const int q = (base + l) >> 1;
                if (q != cur) {
                    if (cur >= 0 && lane == 0) acc[wid][cur] += c;
                    cur = q;
                    c = 0.0;
                }
                const double d = rowdot(cl);
                c += ng ? -d : d;
            }
            if (cur >= 0 && lane == 0) acc[wid][cur] += c;
        }
        const double d = SYM ? 0.5 * rowdot(r) : rowdot(r);
        if (lane == 0) {
            for (int i = 0; i < no; i++) {
                const double nu = (double)((up >> i) & 1u), nd = (double)((dn >> i) & 1u);
                acc[wid][nb + i] += nu * nd * d;
                acc[wid][nb + no + i] += (nu + nd) * d;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += 64 * kCWaves) {
        double sum = 0.0;
        for (int w = 0; w < kCWaves; w++) sum += acc[w][i];
        part[(int64_t)i * gridDim.x + blockIdx.x] = sum;
    }
}

template <typename T, bool SYM = false>
static void launch_contract_rows(unsigned g, hipStream_t s, int64_t n, const mcd_op *op,
                                 const T *L, int KP, const T *Rt, int S, double *part,
                                 int pl = 0) {
#define CR(NRV)                                                                             \
    hipLaunchKernelGGL((k_contract_rows<T, NRV, SYM>), dim3(g), dim3(64 * kCWaves), 0, s, n, \
                       op->d_keys, op->d_model, op->d_hash, op->hash_mask, L, KP, pl, Rt, S,  \
                       part)
    const int nr = S / 64;
    if (nr <= 2) CR(2);
    else if (nr <= 4) CR(4);
    else if (nr <= 6) CR(6);
    else if (nr <= 8) CR(8);
    else if (nr <= 12) CR(12);
    else if (nr <= 16) CR(16);
    else if (nr <= 24) CR(24);
    else if (nr <= 32) CR(32);
    else CR(0);
#undef CR
}

// out[p] (+)= sum_c part[p * nblk + c]: one wavefront per parameter.
__global__ __launch_bounds__(256) void k_param_reduce(int np, int nblk,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ out, int accumulate) {
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= np) return;
    double s = 0.0;
    for (int c = lane; c < nblk; c += 64) s += part[(int64_t)p * nblk + c];
    s = wave_sum(s);
    if (lane == 0) out[p] = accumulate ? out[p] + s : s;
}

// Conjugate-gradient vector updates (scalars from the host).
// (The solve's scalars stay on the device: each kernel reads them there.)
// y = y - e0 x - c psi, c = *c_dev.
__global__ void k_shift_project(int64_t n, double *__restrict__ y, const double *__restrict__ x,
                                double e0, const double *__restrict__ psi,
                                const double *__restrict__ c_dev) {
    const double c = *c_dev;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) y[r] = y[r] - e0 * x[r] - c * psi[r];
}
// x += a p, res -= a ap with a = *rr / *pap (rr = <res, z>, z the
// preconditioned residual); nothing when pap <= 0 (the solve stops there).
__global__ void k_axpy2(int64_t n, const double *__restrict__ rr, const double *__restrict__ pap,
                        const double *__restrict__ p, const double *__restrict__ ap,
                        double *__restrict__ x, double *__restrict__ res) {
    if (!(*pap > 0.0)) return;
    const double a = *rr / *pap;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    x[r] += a * p[r];
    res[r] -= a * ap[r];
}
// y = x + b y with b = *rr2 / *rr.
__global__ void k_xpby(int64_t n, const double *__restrict__ x, const double *__restrict__ rr2,
                       const double *__restrict__ rr, double *__restrict__ y) {
    const double b = *rr2 / *rr;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) y[r] = x[r] + b * y[r];
}
__global__ void k_sub_scaled(int64_t n, double *__restrict__ y, double c,
                             const double *__restrict__ x) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) y[r] -= c * x[r];
}
// Jacobi step of the preconditioned solve: z = r / max(d - e0, dfloor) (d the
// diagonal of H) and the workgroup partials of <psi, z>; grid-stride, fixed
// order.
__global__ __launch_bounds__(BS) void k_jacobi(int64_t n, const double *__restrict__ r,
                                               const double *__restrict__ d, double e0,
                                               double dfloor, const double *__restrict__ psi,
                                               double *__restrict__ z,
                                               double *__restrict__ partials) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BS) {
        const double v = r[i] / fmax(d[i] - e0, dfloor);
        z[i] = v;
        acc += psi[i] * v;
    }
    store_partial<BS>(block_sum<BS>(acc), partials);
}
// z -= c psi (c = *c_dev) and the workgroup partials of <r, z>.
__global__ __launch_bounds__(BS) void k_project_dot(int64_t n, double *__restrict__ z,
                                                    const double *__restrict__ psi,
                                                    const double *__restrict__ c_dev,
                                                    const double *__restrict__ r,
                                                    double *__restrict__ partials) {
    const double c = *c_dev;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BS) {
        const double v = z[i] - c * psi[i];
        z[i] = v;
        acc += r[i] * v;
    }
    store_partial<BS>(block_sum<BS>(acc), partials);
}

// First block column of (z - T)^-1 times R0 (first p columns) for the block
// tridiagonal T of a run: x_0 = S_0^-1 R0, x_j = S_j^-1 B_j x_{j-1}, with the
// Schur complements S_{m-1} = z - A_{m-1}, S_j = z - A_j - B_{j+1}^T
// S_{j+1}^-1 B_{j+1} (the same recursion as block_cf).  X: [m P][p].
static void block_solve_first(const BandResult &br, cplx z, int p, std::vector<cplx> &X) {
    const int P = br.P, m = br.m;
    std::vector<std::vector<cplx>> S(m, std::vector<cplx>(P * P));
    auto zA = [&](int j, std::vector<cplx> &out) {
        for (int a = 0; a < P; a++)
            for (int b = 0; b < P; b++)
                out[a * P + b] = (a == b ? z : cplx(0.0)) - br.A[j][a * P + b];
    };
    zA(m - 1, S[m - 1]);
    for (int j = m - 2; j >= 0; j--) {
        std::vector<cplx> Y(P * P), Sc = S[j + 1];
        for (int e = 0; e < P * P; e++) Y[e] = br.B[j + 1][e];
        csolve(P, P, Sc, Y);
        zA(j, S[j]);
        for (int a = 0; a < P; a++)
            for (int b = 0; b < P; b++) {
                cplx acc = 0.0;
                for (int q = 0; q < P; q++) acc += br.B[j + 1][q * P + a] * Y[q * P + b];
                S[j][a * P + b] -= acc;
            }
    }
    X.assign((size_t)m * P * p, cplx(0.0));
    std::vector<cplx> rhs(P * p);
    for (int a = 0; a < P; a++)
        for (int b = 0; b < p; b++) rhs[a * p + b] = br.R0[a * P + b];
    for (int j = 0; j < m; j++) {
        if (j > 0) {
            for (int a = 0; a < P; a++)
                for (int b = 0; b < p; b++) {
                    cplx acc = 0.0;
                    for (int q = 0; q < P; q++)
                        acc += br.B[j][a * P + q] * X[((size_t)(j - 1) * P + q) * p + b];
                    rhs[a * p + b] = acc;
                }
        }
        std::vector<cplx> Sc = S[j];
        csolve(P, p, Sc, rhs);
        for (int a = 0; a < P; a++)
            for (int b = 0; b < p; b++) X[((size_t)j * P + a) * p + b] = rhs[a * p + b];
    }
}

template <typename T>
static int band_green_vjp(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                          const double *psi0_dev, double e0, const SelOps &sel, int n_freq,
                          const double *omega, const mcd_band_cfg *cfg, const double *G_bar,
                          double e0_bar, double cg_tol, int cg_max_iter, double *d_t,
                          double *d_U, double *d_eps, mcd_solve_info *info, mcd_ws *ws,
                          hipStream_t s, Instance<T> *keep = nullptr) {
    const Alloc A{ws};
    const double t0 = wall_ms();
    const int p = sel.n;
    int P = 1;
    while (P < p) P <<= 1;
    mcd_op *op_gs = nullptr;
    double *lam = nullptr, *acc = nullptr, *part = nullptr, *scal = nullptr;
    double *xi = nullptr, *res = nullptr, *dir = nullptr, *adir = nullptr;
    double *psi_n = nullptr, *scr = nullptr, *zv = nullptr;
    Instance<T> rec;   // the recomputed sector runs (without a kept forward)
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);   // queued work reads the pieces
        rec.plus.release();
        rec.minus.release();
        for (void *q : {(void *)zv, (void *)adir, (void *)dir, (void *)res, (void *)xi,
                        (void *)part, (void *)scal, (void *)acc, (void *)lam, (void *)scr,
                        (void *)psi_n})
            if (q) (void)dfree(q, A);
        if (op_gs) mcd_op_destroy(op_gs);
        op_gs = nullptr;
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
#define TRY(expr)          \
    do {                   \
        int rc_ = (expr);  \
        if (rc_ < 0) {     \
            cleanup();     \
            return rc_;    \
        }                  \
    } while (0)
    // untuned: the default row-ordered product kernel, so that the solve (and
    // the derivative) is reproducible bit for bit across calls
    TRY(op_create(model, keys_dev, n, MCD_STORAGE_AUTO, 0, false, ws, s, &op_gs));
    const int nb = op_gs->hm.dm.n_bonds, no = op_gs->hm.dm.n_orb, np = nb + 2 * no;
    // psi0 normalised exactly as the forward call does, so the band runs below
    // reproduce the forward's recurrence (and stopping point) bit for bit
    CK(dmalloc((void **)&psi_n, n * sizeof(double), A));
    CK(dmalloc((void **)&scr, (4096 + 8) * sizeof(double), A));
    CK(poison_fp(psi_n, n * sizeof(double), A, s));
    CK(poison_fp(scr, (4096 + 8) * sizeof(double), A, s));
    CK(hipMemcpyAsync(psi_n, psi0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    {
        const unsigned nbn = std::min<unsigned>(gridn(n, BS), 2048);
        hipLaunchKernelGGL(k_norm2, dim3(nbn), dim3(BS), 0, s, n, psi_n, scr);
        hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)nbn, scr,
                           scr + 4096);
        hipLaunchKernelGGL(k_scale_by, dim3(gridn(n, 256)), dim3(256), 0, s, n, psi_n,
                           scr + 4096);
        CK(hipGetLastError());
    }
    CK(dmalloc((void **)&lam, n * sizeof(double), A));
    CK(dmalloc((void **)&acc, np * sizeof(double), A));
    CK(dmalloc((void **)&scal, 8 * sizeof(double), A));
    CK(poison_fp(lam, n * sizeof(double), A, s));
    CK(poison_fp(acc, np * sizeof(double), A, s));
    CK(poison_fp(scal, 8 * sizeof(double), A, s));
    CK(hipMemsetAsync(lam, 0, n * sizeof(double), s));
    CK(hipMemsetAsync(acc, 0, np * sizeof(double), s));
    const int cblk = 16384;   // contraction workgroups at most (partials per parameter)
    CK(dmalloc((void **)&part, (size_t)np * cblk * sizeof(double), A));
    CK(poison_fp(part, (size_t)np * cblk * sizeof(double), A, s));

    double trM = 0.0;   // sum over sectors of tr(M)
    int krylov = 0;
    const int reorth = std::max(0, std::min(2, (int)cfg->reorth));
    const int fb = cfg->vjp_freq_batch > 0 ? std::min<int>(cfg->vjp_freq_batch, n_freq) : n_freq;
    // Default chunk: as many Krylov vectors as the work matrices U, V have
    // columns (a chunk buffer no larger than U), at least 16 blocks; each
    // flush reads and writes U and V once, so fewer flushes move less.
    const int chunk = cfg->vjp_chunk > 0
                          ? cfg->vjp_chunk
                          : std::max(16, ((2 * fb * p + 127) / 128 * 128) / std::max(P, 1));
    // Without kept runs and without reorthogonalisation no Krylov block is
    // stored: a second pass of the recurrence (the same kernels on the same
    // data) regenerates Q_0, Q_1, ... one at a time.
    const bool streaming = keep == nullptr && reorth == 0;
    int pl = 0;
    while ((1 << pl) < P) pl++;

    // Per sector, on the host: the per-frequency solves give Omega and the
    // two factors of M = sg A B^T (A, B: KP x K2, K2 = 2 n_freq p).
    struct SectorPrep {
        int m = 0, KP = 0;
        double sg = 1.0;
        std::vector<double> Om, Am, Bm;
    };
    auto prep = [&](const BandRun<T> &run, bool create, SectorPrep &sp) {
        const BandResult &br = run.br;
        const int m = br.m, KP = m * P;
        const double sg = create ? 1.0 : -1.0;
        sp.m = m;
        sp.KP = KP;
        sp.sg = sg;
        std::vector<double> &Om = sp.Om;
        Om.assign((size_t)KP * P, 0.0);
        // Per frequency (in parallel): X_f = first block column of
        // (z - T)^-1 R0, V_f = X_f conj(G_bar_f)^T.  Then M and Omega
        // (in parallel over their rows a), each element summed over the
        // frequencies in index order.
        std::vector<std::vector<cplx>> Xs(n_freq), Vs(n_freq);
        std::vector<std::vector<double>> Ws(n_freq);
        parallel_for(n_freq, [&](int f) {
            const cplx zeta = freq_arg(cfg, omega[f]);
            block_solve_first(br, create ? e0 + zeta : e0 - zeta, p, Xs[f]);
            const std::vector<cplx> &X = Xs[f];
            std::vector<cplx> &V = Vs[f];
            std::vector<double> &Wf = Ws[f];
            V.assign((size_t)KP * p, cplx(0.0));
            Wf.assign((size_t)KP * p, 0.0);
            const cplx *Gb = (const cplx *)G_bar + (size_t)f * p * p;
            for (int a = 0; a < KP; a++)
                for (int mu = 0; mu < p; mu++) {
                    cplx v = 0.0, w = 0.0;
                    for (int nu = 0; nu < p; nu++) {
                        v += X[(size_t)a * p + nu] * std::conj(Gb[mu * p + nu]);
                        w += X[(size_t)a * p + nu] * std::conj(Gb[nu * p + mu]);
                    }
                    V[(size_t)a * p + mu] = v;
                    Wf[(size_t)a * p + mu] = (v + w).real();
                }
        });
        // M[a][b] = sg Re sum_f sum_mu V_f[a][mu] X_f[b][mu] as a real
        // product A B^T over K2 = 2 n_freq p terms: A[a] = (Re V, -Im V),
        // B[b] = (Re X, Im X), contiguous per row.  M itself is never
        // formed: the device makes Q A and Q B below; the host keeps tr(M).
        const int K2 = 2 * n_freq * p;
        std::vector<double> &Am = sp.Am, &Bm = sp.Bm;
        Am.assign((size_t)KP * K2, 0.0);
        Bm.assign((size_t)KP * K2, 0.0);
        parallel_for(KP, [&](int a) {
            double *Aa = Am.data() + (size_t)a * K2, *Ba = Bm.data() + (size_t)a * K2;
            for (int f = 0; f < n_freq; f++)
                for (int mu = 0; mu < p; mu++) {
                    const cplx v = Vs[f][(size_t)a * p + mu], x = Xs[f][(size_t)a * p + mu];
                    const size_t k = 2 * ((size_t)f * p + mu);
                    Aa[k] = v.real();
                    Aa[k + 1] = -v.imag();
                    Ba[k] = x.real();
                    Ba[k + 1] = x.imag();
                }
        });
        std::vector<double> diag(KP);
        parallel_for(KP, [&](int a) {
            for (int f = 0; f < n_freq; f++)
                for (int mu = 0; mu < p; mu++)
                    Om[(size_t)a * P + mu] += sg * Ws[f][(size_t)a * p + mu];
            const double *Aa = Am.data() + (size_t)a * K2, *Ba = Bm.data() + (size_t)a * K2;
            double t = 0.0;
            for (int k = 0; k < K2; k++) t += Aa[k] * Ba[k];
            diag[a] = sg * t;
        });
        for (int a = 0; a < KP; a++) trM += diag[a];
        krylov += br.krylov;
    };

    // Per sector without a store (the blocks regenerated), on the device, for
    // each batch of frequencies: over chunks of Krylov blocks Q_c,
    //   U += Q_c (sg A_c),  V += Q_c B_c  (columns of the batch),
    //   W += Q_c Omega_c                  (first batch),
    // then tr(Q^T dH Q M) restricted to the batch = tr(U^T dH V) into acc
    // (M = sg A B^T and dH symmetric); finally lam += (start-block map)^T W.
    auto sector = [&](BandRun<T> &run, bool create, const SectorPrep &sp) -> int {
        const mcd_op *op = run.op;
        const int m = sp.m, KP = sp.KP;
        const int64_t nx = run.n;
        const int K2 = 2 * n_freq * p;
        const int nbatch = (n_freq + fb - 1) / fb;
        const int S2 = (2 * fb * p + 127) / 128 * 128;
        const int KPr = KP + 64;   // coefficient rows (zero past KP; read up to 32 past a chunk)
        constexpr int kTail = 1024;   // zeroed values after the last row of U and V
        Arena za(ws);
        T *U = nullptr, *V = nullptr, *Wo = nullptr, *dA = nullptr, *dB = nullptr, *Qc = nullptr;
        double *dC = nullptr;
        int rc = MCD_OK;
        auto get = [&](void **ptr, size_t bytes) {
            if (rc != MCD_OK) return;
            if (za.get(ptr, bytes) != hipSuccess) {
                set_error("green vjp: workspace too small for the contraction matrices "
                          "(%.2f GB more; lower vjp_freq_batch)", bytes / 1e9);
                rc = MCD_E_WORKSPACE;
            } else if (poison_fp(*ptr, bytes, za.al, s) != hipSuccess) {
                rc = MCD_E_HIP;
            }
        };
        get((void **)&U, ((size_t)nx * S2 + kTail) * sizeof(T));
        get((void **)&V, ((size_t)nx * S2 + kTail) * sizeof(T));
        get((void **)&Wo, (size_t)nx * P * sizeof(T));
        get((void **)&dA, (size_t)KPr * S2 * sizeof(T));
        get((void **)&dB, (size_t)KPr * S2 * sizeof(T));
        get((void **)&dC, (size_t)m * P * P * sizeof(double));
        get((void **)&Qc, (size_t)chunk * nx * P * sizeof(T));
        std::vector<double> C((size_t)m * P * P);
        for (size_t e = 0; e < C.size(); e++) C[e] = -sp.Om[e];   // W -= Q (-Omega)
        std::vector<T> hA((size_t)KPr * S2), hB((size_t)KPr * S2);
        if (rc == MCD_OK &&
            (hipMemcpyAsync(dC, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s) !=
                 hipSuccess ||
             hipMemsetAsync(Wo, 0, (size_t)nx * P * sizeof(T), s) != hipSuccess))
            rc = MCD_E_HIP;
        const unsigned g =
            (unsigned)std::min<int64_t>(cblk, (nx + 16 * kCWaves - 1) / (16 * kCWaves));
        const int64_t tiles = (nx + 127) / 128 * (S2 / 128);
        const unsigned gt = (unsigned)((tiles + 7) / 8 * 8);
        for (int b = 0; b < nbatch && rc == MCD_OK; b++) {
            const int f0 = b * fb, f1 = std::min(n_freq, f0 + fb);
            const int K2b = 2 * (f1 - f0) * p;
            std::fill(hA.begin(), hA.end(), (T)0);
            std::fill(hB.begin(), hB.end(), (T)0);
            parallel_for(KP, [&](int a) {
                const double *Aa = sp.Am.data() + (size_t)a * K2 + 2 * (size_t)f0 * p;
                const double *Ba = sp.Bm.data() + (size_t)a * K2 + 2 * (size_t)f0 * p;
                for (int k = 0; k < K2b; k++) {
                    hA[(size_t)a * S2 + k] = (T)(sp.sg * Aa[k]);
                    hB[(size_t)a * S2 + k] = (T)Ba[k];
                }
            });
            if (hipMemcpyAsync(dA, hA.data(), hA.size() * sizeof(T), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                hipMemcpyAsync(dB, hB.data(), hB.size() * sizeof(T), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                hipMemsetAsync(U, 0, ((size_t)nx * S2 + kTail) * sizeof(T), s) != hipSuccess ||
                hipMemsetAsync(V, 0, ((size_t)nx * S2 + kTail) * sizeof(T), s) != hipSuccess) {
                rc = MCD_E_HIP;
                break;
            }
            // the k blocks at Qp (consecutive) are blocks j0 .. j0 + k - 1
            auto flush = [&](const T *Qp, int j0, int k) -> int {
                hipLaunchKernelGGL((k_rows_times<T>), dim3(gt), dim3(256), 0, s, nx, S2, k * P, pl,
                                   Qp, dA + (size_t)j0 * P * S2, U);
                hipLaunchKernelGGL((k_rows_times<T>), dim3(gt), dim3(256), 0, s, nx, S2, k * P, pl,
                                   Qp, dB + (size_t)j0 * P * S2, V);
                MCD_HIP(hipGetLastError());
                if (b == 0) MCD_TRY(run.block_apply_dev(Qp, k, dC + (size_t)j0 * P * P, Wo, true));
                return MCD_OK;
            };
            // the cut, the start block and the recurrence again, capped at
            // the first pass's m blocks; each new block is copied to the
            // chunk buffer before the ring reuses its slot
            uint64_t *kt = nullptr;
            double *pt = nullptr;
            int64_t nk = 0;
            rc = wt_cut(keys_dev, n, psi0_dev, cfg->w_t, ws, s, &kt, &pt, &nk);
            if (rc == MCD_OK) rc = run_start_block(run, kt, pt, nk, sel, create);
            (void)dfree(pt, A);
            (void)dfree(kt, A);
            int cnt = 0, jn = 0;
            BlockHook<T> hk = [&](BandRun<T> &r, int j) -> int {
                if (j >= m) return MCD_OK;
                MCD_HIP(hipMemcpyAsync(Qc + (size_t)cnt * nx * P, r.blk(j),
                                       (size_t)nx * P * sizeof(T), hipMemcpyDeviceToDevice, s));
                cnt++;
                if (cnt == chunk || j == m - 1) {
                    MCD_TRY(flush(Qc, jn, cnt));
                    jn += cnt;
                    cnt = 0;
                }
                return MCD_OK;
            };
            const double gtol = run.g_tol;
            run.g_tol = 0.0;
            run.limit = m;
            std::vector<BandRun<T> *> one{&run};
            if (rc == MCD_OK) rc = run_lockstep<T>(one, cfg->dtol, 0, s, &hk);
            run.g_tol = gtol;
            run.limit = 0;
            if (rc == MCD_OK && (run.br.m != m || jn != m)) {
                set_error("green vjp: the regenerated Krylov blocks (%d) differ from the "
                          "first pass (%d)", jn, m);
                rc = MCD_E_NUMERIC;
            }
            if (rc == MCD_OK) {
                launch_contract_rows<T>(g, s, nx, op, U, K2b, V, S2, part);
                hipLaunchKernelGGL(k_param_reduce, dim3((np + 3) / 4), dim3(256), 0, s, np, (int)g,
                                   part, acc, 1);
                if (hipGetLastError() != hipSuccess) rc = MCD_E_HIP;
            }
        }
        if (rc == MCD_OK) {
            hipLaunchKernelGGL((k_start_block_t<T>), dim3(gridn(n, 256)), dim3(256), 0, s, n,
                               keys_dev, sel, create ? 1 : 0, op->d_hash, op->hash_mask, P, Wo,
                               lam);
            if (hipGetLastError() != hipSuccess) rc = MCD_E_HIP;
        }
        if (hipStreamSynchronize(s) != hipSuccess && rc == MCD_OK) rc = MCD_E_HIP;
        za.release();   // after the synchronisation above
        if (rc == MCD_E_HIP) set_error("green vjp: device step failed in a sector");
        return rc;
    };

    // With every Krylov block stored (kept runs, or a recomputed run with
    // reorthogonalisation) the weight is taken whole: Mp = M + M^T (S x S, S =
    // KP rounded up to 128) from A and B on the device, Z = Q Mp (one MFMA
    // product over the store), then tr(Q^T dH Q M) by the symmetric
    // contraction of the store with Z (each hop pair once), W = Q Omega, and
    // lam += (start-block map)^T W.  Fewer operations than the factored form
    // of the regenerated blocks (one n x S product instead of two n x S2, half
    // the contraction's gathers); the two agree to rounding.
    auto sector_stored = [&](BandRun<T> &run, bool create, const SectorPrep &sp) -> int {
        const mcd_op *op = run.op;
        const int m = sp.m, KP = sp.KP;
        const int64_t nx = run.n;
        const int K2 = 2 * n_freq * p;
        const int S = (KP + 127) / 128 * 128;
        constexpr int kTail = 1024;   // zeroed values after the last row of Z
        Arena za(ws);
        T *Z = nullptr, *Mp = nullptr, *Wo = nullptr;
        double *dA = nullptr, *dB = nullptr, *dC = nullptr;
        int rc = MCD_OK;
        auto get = [&](void **ptr, size_t bytes) {
            if (rc != MCD_OK) return;
            if (za.get(ptr, bytes) != hipSuccess) {
                set_error("green vjp: workspace too small for the contraction matrices "
                          "(%.2f GB more)", bytes / 1e9);
                rc = MCD_E_WORKSPACE;
            } else if (poison_fp(*ptr, bytes, za.al, s) != hipSuccess) {
                rc = MCD_E_HIP;
            }
        };
        get((void **)&Z, ((size_t)nx * S + kTail) * sizeof(T));
        get((void **)&Mp, (size_t)S * S * sizeof(T));
        get((void **)&Wo, (size_t)nx * P * sizeof(T));
        get((void **)&dA, (size_t)KP * K2 * sizeof(double));
        get((void **)&dB, (size_t)KP * K2 * sizeof(double));
        get((void **)&dC, (size_t)m * P * P * sizeof(double));
        std::vector<double> C((size_t)m * P * P);
        for (size_t e = 0; e < C.size(); e++) C[e] = -sp.Om[e];   // W -= Q (-Omega)
        if (rc == MCD_OK &&
            (hipMemcpyAsync(dC, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s) !=
                 hipSuccess ||
             hipMemcpyAsync(dA, sp.Am.data(), (size_t)KP * K2 * sizeof(double),
                            hipMemcpyHostToDevice, s) != hipSuccess ||
             hipMemcpyAsync(dB, sp.Bm.data(), (size_t)KP * K2 * sizeof(double),
                            hipMemcpyHostToDevice, s) != hipSuccess ||
             hipMemsetAsync(Wo, 0, (size_t)nx * P * sizeof(T), s) != hipSuccess ||
             hipMemsetAsync(Z, 0, ((size_t)nx * S + kTail) * sizeof(T), s) != hipSuccess))
            rc = MCD_E_HIP;
        if (rc == MCD_OK) {
            hipLaunchKernelGGL((k_sym_gram<T>), dim3(S / 16, S / 16), dim3(16, 16), 0, s, KP, K2,
                               S, sp.sg, dA, dB, Mp);
            const int64_t tiles = (nx + 127) / 128 * (S / 128);
            hipLaunchKernelGGL((k_rows_times<T>), dim3((unsigned)((tiles + 7) / 8 * 8)),
                               dim3(256), 0, s, nx, S, KP, pl, run.blk(0), Mp, Z);
            if (hipGetLastError() != hipSuccess) rc = MCD_E_HIP;
        }
        if (rc == MCD_OK) rc = run.block_apply_dev(run.blk(0), m, dC, Wo, true);
        if (rc == MCD_OK) {
            const unsigned g =
                (unsigned)std::min<int64_t>(cblk, (nx + 16 * kCWaves - 1) / (16 * kCWaves));
            launch_contract_rows<T, true>(g, s, nx, op, run.blk(0), KP, Z, S, part, pl);
            hipLaunchKernelGGL(k_param_reduce, dim3((np + 3) / 4), dim3(256), 0, s, np, (int)g,
                               part, acc, 1);
            hipLaunchKernelGGL((k_start_block_t<T>), dim3(gridn(n, 256)), dim3(256), 0, s, n,
                               keys_dev, sel, create ? 1 : 0, op->d_hash, op->hash_mask, P, Wo,
                               lam);
            if (hipGetLastError() != hipSuccess) rc = MCD_E_HIP;
        }
        if (hipStreamSynchronize(s) != hipSuccess && rc == MCD_OK) rc = MCD_E_HIP;
        za.release();   // after the synchronisation above
        if (rc == MCD_E_HIP) set_error("green vjp: device step failed in a sector");
        return rc;
    };

    int64_t npl = 0, nmi = 0;
    {
        // the forward call's sector runs, kept, or recomputed here (from psi0
        // as given: the cut normalises it exactly as the forward call does, so
        // the recurrence is the same), every block stored unless streaming
        Instance<T> *src = keep;
        if (!keep) {
            rec.model = model;
            rec.keys = keys_dev;
            rec.n = n;
            rec.psi = psi0_dev;
            rec.e0 = e0;
            std::vector<Instance<T> *> one{&rec};
            TRY(band_green_multi<T>(one, sel, n_freq, omega, cfg, ws, s, !streaming, nullptr,
                                    true, nullptr));
            src = &rec;
        }
        npl = src->plus.n;
        nmi = src->minus.n;
        for (int side = 0; side < 2; side++) {
            BandRun<T> &r = side == 0 ? src->plus : src->minus;
            if (r.br.m > 0 && r.op) {
                SectorPrep sp;
                prep(r, side == 0, sp);
                const hipStream_t s_prev = r.s;
                r.s = s;
                const int rc_h =
                    streaming ? sector(r, side == 0, sp) : sector_stored(r, side == 0, sp);
                r.s = s_prev;
                TRY(rc_h);
            }
        }
        rec.plus.release();
        rec.minus.release();
    }

    // (H - E0) xi = P lam on F~, xi orthogonal to psi0: conjugate gradients
    // (H - E0 is positive definite on the complement of a non-degenerate
    // psi0), preconditioned by P D^-1 P with D = diag(H) - E0 (Jacobi; D >= 0
    // since E0 is at most any diagonal element, floored for safety).
    CK(dmalloc((void **)&xi, n * sizeof(double), A));
    CK(dmalloc((void **)&res, n * sizeof(double), A));
    CK(dmalloc((void **)&dir, n * sizeof(double), A));
    CK(dmalloc((void **)&adir, n * sizeof(double), A));
    CK(dmalloc((void **)&zv, n * sizeof(double), A));
    for (double *v : {xi, res, dir, adir, zv}) CK(poison_fp(v, n * sizeof(double), A, s));
    const unsigned gv = gridn(n, 256);
    const unsigned gp = std::min<unsigned>(gridn(n, BS), 2048);   // partial-sum kernels
    const double dfloor = 1e-6 * std::max(1.0, fabs(e0));
    auto dot = [&](const double *a, const double *b, double *out) -> int {
        MCD_TRY(dev_dot(op_gs, a, b, n, scal, s));
        MCD_HIP(hipMemcpyAsync(out, scal, sizeof(double), hipMemcpyDeviceToHost, s));
        MCD_HIP(hipStreamSynchronize(s));
        return MCD_OK;
    };
    // zv = P D^-1 res, *rz_d = <res, zv> (scal[6] holds <psi0, D^-1 res>)
    auto precond = [&](double *rz_d) -> int {
        hipLaunchKernelGGL(k_jacobi, dim3(gp), dim3(BS), 0, s, n, res, op_gs->d_diag, e0, dfloor,
                           psi_n, zv, op_gs->d_partials);
        hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)gp,
                           op_gs->d_partials, scal + 6);
        hipLaunchKernelGGL(k_project_dot, dim3(gp), dim3(BS), 0, s, n, zv, psi_n, scal + 6, res,
                           op_gs->d_partials);
        hipLaunchKernelGGL((k_finalize_sum<BS>), dim3(1), dim3(BS), 0, s, (int)gp,
                           op_gs->d_partials, rz_d);
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    };
    double c = 0.0;
    CK(hipMemcpyAsync(res, lam, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    TRY(dot(psi_n, res, &c));
    hipLaunchKernelGGL(k_sub_scaled, dim3(gv), dim3(256), 0, s, n, res, c, psi_n);
    CK(hipMemsetAsync(xi, 0, n * sizeof(double), s));
    // device scalars: scal[1] = <psi0, A dir>, scal[2] = <dir, A dir>,
    // scal[3 + (it & 1)] = <res, z> at the start of iteration it, scal[5] =
    // <res, res>; the host reads pap and <res, res> once per iteration
    double rr = 0.0;
    TRY(dev_dot(op_gs, res, res, n, scal + 5, s));
    TRY(precond(scal + 3));
    CK(hipMemcpyAsync(dir, zv, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(&rr, scal + 5, sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (!std::isfinite(rr)) {
        cleanup();
        set_error("green vjp: non-finite right-hand side of the response solve");
        return MCD_E_NUMERIC;
    }
    const double bnorm = sqrt(rr);
    int it = 0;
    bool conv = bnorm == 0.0;
    double rel = 0.0;
    while (!conv && it < cg_max_iter) {
        double *rz_d = scal + 3 + (it & 1), *rz2_d = scal + 3 + ((it + 1) & 1);
        TRY(apply_any(op_gs, MCD_F64, 1, dir, adir, s));
        TRY(dev_dot(op_gs, psi_n, adir, n, scal + 1, s));
        hipLaunchKernelGGL(k_shift_project, dim3(gv), dim3(256), 0, s, n, adir, dir, e0, psi_n,
                           scal + 1);
        TRY(dev_dot(op_gs, dir, adir, n, scal + 2, s));
        hipLaunchKernelGGL(k_axpy2, dim3(gv), dim3(256), 0, s, n, rz_d, scal + 2, dir, adir, xi,
                           res);
        TRY(dev_dot(op_gs, res, res, n, scal + 5, s));
        TRY(precond(rz2_d));
        double pap = 0.0, rr2 = 0.0;
        CK(hipMemcpyAsync(&pap, scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(&rr2, scal + 5, sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        if (!std::isfinite(pap) || !std::isfinite(rr2)) {
            cleanup();
            set_error("green vjp: non-finite value in the response solve (iteration %d)", it);
            return MCD_E_NUMERIC;
        }
        if (!(pap > 0.0)) {   // not positive definite: psi0 is no non-degenerate ground state
            cleanup();
            set_error("green vjp: the response solve met <p, (H - E0) p> = %g <= 0 at iteration "
                      "%d (psi0 is not a non-degenerate ground state of H~)", pap, it);
            return MCD_E_BREAKDOWN;
        }
        it++;
        rel = sqrt(rr2) / bnorm;
        if (rel <= cg_tol) {
            conv = true;
            break;
        }
        hipLaunchKernelGGL(k_xpby, dim3(gv), dim3(256), 0, s, n, zv, rz2_d, rz_d, dir);
    }
    CK(hipGetLastError());
    // contractions with psi0: dE0 and <xi| dH |psi0>
    const int nlb = model->n_bonds;
    std::vector<double> e_t(nlb), e_U(no), e_e(no), x_t(nlb), x_U(no), x_e(no);
    TRY(mcd_hamiltonian_contract(op_gs, model, psi_n, psi_n, e_t.data(), e_U.data(),
                                 e_e.data(), ws, s));
    TRY(mcd_hamiltonian_contract(op_gs, model, xi, psi_n, x_t.data(), x_U.data(), x_e.data(),
                                 ws, s));
    std::vector<double> h(np);
    CK(hipMemcpyAsync(h.data(), acc, np * sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const double ce = e0_bar - trM;
    for (int q = 0; q < nlb; q++) {
        const int i = std::min(model->bond_i[q], model->bond_j[q]);
        const int j = std::max(model->bond_i[q], model->bond_j[q]);
        const uint32_t mask = (1u << i) | (1u << j);
        double v = 0.0;
        for (int mb = 0; mb < nb; mb++)
            if (op_gs->hm.dm.bonds[mb].mask == mask) v = h[mb];
        if (d_t) d_t[q] = v + ce * e_t[q] - x_t[q];
    }
    for (int i = 0; i < no; i++) {
        if (d_U) d_U[i] = h[nb + i] + ce * e_U[i] - x_U[i];
        if (d_eps) d_eps[i] = h[nb + no + i] + ce * e_e[i] - x_e[i];
    }
    cleanup();
#undef CK
#undef TRY
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = it;
        info->converged = conv ? 1 : 0;
        info->e0 = e0;
        info->residual = rel;
        info->solve_ms = wall_ms() - t0;
        info->krylov_dim = krylov;
        info->n_plus = npl;
        info->n_minus = nmi;
        info->n_truncated = n;
    }
    return conv ? MCD_OK : MCD_NOCONV;
}

}  // namespace mcd

using namespace mcd;

// Checks of the forward call's arguments; fills sel.
static int band_args(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                     const double *psi0_dev, int32_t n_sel, const int32_t *orb,
                     const int32_t *spin, int32_t n_freq, const double *omega,
                     const mcd_band_cfg *cfg, const double *G_out, SelOps &sel) {
    MCD_REQUIRE(model && cfg && keys_dev && psi0_dev && orb && spin && G_out, MCD_E_INVALID,
                "a required pointer is NULL");
    MCD_REQUIRE(n >= 1, MCD_E_INVALID, "empty basis");
    MCD_REQUIRE(n_sel >= 1 && n_sel <= 16, MCD_E_INVALID, "n_sel = %d outside 1..16", n_sel);
    MCD_REQUIRE(n_freq >= 0 && (n_freq == 0 || omega), MCD_E_INVALID, "bad frequencies");
    MCD_REQUIRE(cfg->w_t > 0.0 && cfg->w_t <= 1.0, MCD_E_INVALID, "w_t must be in (0, 1]");
    MCD_REQUIRE(cfg->max_blocks >= 1, MCD_E_INVALID, "max_blocks must be >= 1");
    MCD_REQUIRE(cfg->precision == MCD_F64 || cfg->precision == MCD_F32, MCD_E_INVALID,
                "precision must be MCD_F64 or MCD_F32");
    HostModel hm;
    MCD_TRY(prepare_model(model, &hm));
    memset(&sel, 0, sizeof(sel));
    sel.n = n_sel;
    for (int q = 0; q < n_sel; q++) {
        MCD_REQUIRE(orb[q] >= 0 && orb[q] < model->n_orb && (spin[q] == 0 || spin[q] == 1),
                    MCD_E_INVALID, "selection %d = (%d, %d) invalid", q, orb[q], spin[q]);
        sel.orb[q] = orb[q];
        sel.spin[q] = spin[q];
    }
    return MCD_OK;
}

// What a kept forward call was made with, and its two sector runs (their
// operators and blocks stay in the forward call's workspace).
struct mcd_band_keep {
    int64_t n = 0;
    int32_t n_sel = 0, orb[16] = {}, spin[16] = {};
    double e0 = 0.0;
    mcd_band_cfg cfg{};
    std::vector<double> omega;
    std::unique_ptr<mcd::Instance<float>> kf;
    std::unique_ptr<mcd::Instance<double>> kd;
};

template <typename T>
static int band_one(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                    const double *psi0_dev, double e0, const SelOps &sel, int32_t n_freq,
                    const double *omega, const mcd_band_cfg *cfg, double *G_out, double *Gp_out,
                    double *Gm_out, mcd_solve_info *info, mcd_ws *ws, hipStream_t s,
                    size_t *plan_need, Instance<T> *keep) {
    Instance<T> local;
    Instance<T> &in = keep ? *keep : local;
    in.model = model;
    in.keys = keys_dev;
    in.n = n;
    in.psi = psi0_dev;
    in.e0 = e0;
    in.G_out = G_out;
    in.Gp_out = Gp_out;
    in.Gm_out = Gm_out;
    std::vector<Instance<T> *> one{&in};
    return band_green_multi<T>(one, sel, n_freq, omega, cfg, ws, s, keep != nullptr, plan_need,
                               keep != nullptr, info);
}

extern "C" int mcd_band_lanczos_green(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                                      const double *psi0_dev, double e0, int32_t n_sel,
                                      const int32_t *orb, const int32_t *spin, int32_t n_freq,
                                      const double *omega, const mcd_band_cfg *cfg,
                                      double *G_out, double *Gp_out, double *Gm_out,
                                      mcd_solve_info *info, mcd_ws *ws, void *stream) {
    SelOps sel;
    MCD_TRY(band_args(model, keys_dev, n, psi0_dev, n_sel, orb, spin, n_freq, omega, cfg, G_out,
                      sel));
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (cfg->precision == MCD_F64)
        return band_one<double>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, cfg, G_out,
                                Gp_out, Gm_out, info, ws, s, nullptr, nullptr);
    return band_one<float>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, cfg, G_out,
                           Gp_out, Gm_out, info, ws, s, nullptr, nullptr);
}

extern "C" int mcd_band_workspace_size(const mcd_model *model, const uint64_t *keys_dev,
                                       int64_t n, const double *psi0_dev, double e0,
                                       int32_t n_sel, const int32_t *orb, const int32_t *spin,
                                       int32_t n_freq, const double *omega,
                                       const mcd_band_cfg *cfg, int32_t keep, mcd_ws *ws,
                                       void *stream, size_t *bytes) {
    MCD_REQUIRE(bytes != nullptr, MCD_E_INVALID, "bytes is NULL");
    *bytes = 0;
    SelOps sel;
    double g_dummy = 0.0;
    MCD_TRY(band_args(model, keys_dev, n, psi0_dev, n_sel, orb, spin, n_freq, omega, cfg,
                      &g_dummy, sel));
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "probe workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    const mcd_band_cfg c = *cfg;
    int rc;
    if (cfg->precision == MCD_F64) {
        Instance<double> in;
        rc = band_one<double>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, &c, nullptr,
                              nullptr, nullptr, nullptr, ws, s, bytes, keep ? &in : nullptr);
    } else {
        Instance<float> in;
        rc = band_one<float>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, &c, nullptr,
                             nullptr, nullptr, nullptr, ws, s, bytes, keep ? &in : nullptr);
    }
    return rc;
}

extern "C" int mcd_band_lanczos_green_keep(const mcd_model *model, const uint64_t *keys_dev,
                                           int64_t n, const double *psi0_dev, double e0,
                                           int32_t n_sel, const int32_t *orb,
                                           const int32_t *spin, int32_t n_freq,
                                           const double *omega, const mcd_band_cfg *cfg,
                                           double *G_out, double *Gp_out, double *Gm_out,
                                           mcd_solve_info *info, mcd_ws *ws, void *stream,
                                           mcd_band_keep **keep_out) {
    MCD_REQUIRE(keep_out, MCD_E_INVALID, "keep_out is NULL");
    *keep_out = nullptr;
    SelOps sel;
    MCD_TRY(band_args(model, keys_dev, n, psi0_dev, n_sel, orb, spin, n_freq, omega, cfg, G_out,
                      sel));
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "workspace is NULL");
    MCD_REQUIRE(cfg->w_t >= 1.0, MCD_E_INVALID, "a kept run needs w_t = 1 (no weight cut)");
    MCD_REQUIRE(cfg->per_column == 0, MCD_E_INVALID, "a kept run uses block products");
    std::unique_ptr<mcd_band_keep> k(new mcd_band_keep());
    k->n = n;
    k->n_sel = n_sel;
    for (int q = 0; q < n_sel; q++) {
        k->orb[q] = orb[q];
        k->spin[q] = spin[q];
    }
    k->e0 = e0;
    k->cfg = *cfg;
    k->omega.assign(omega, omega + n_freq);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (cfg->precision == MCD_F64) {
        k->kd.reset(new Instance<double>());
        rc = band_one<double>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, cfg, G_out,
                              Gp_out, Gm_out, info, ws, s, nullptr, k->kd.get());
    } else {
        k->kf.reset(new Instance<float>());
        rc = band_one<float>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, cfg, G_out,
                             Gp_out, Gm_out, info, ws, s, nullptr, k->kf.get());
    }
    if (rc < 0) return rc;   // k and whatever it holds are released
    *keep_out = k.release();
    return rc;
}

extern "C" void mcd_band_keep_destroy(mcd_band_keep *keep) { delete keep; }

static int band_vjp_entry(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                          const double *psi0_dev, double e0, int32_t n_sel, const int32_t *orb,
                          const int32_t *spin, int32_t n_freq, const double *omega,
                          const mcd_band_cfg *cfg, const double *G_bar, double e0_bar,
                          double cg_tol, int32_t cg_max_iter, double *d_t, double *d_U,
                          double *d_eps, mcd_solve_info *info, mcd_ws *ws, void *stream,
                          mcd_band_keep *keep) {
    MCD_REQUIRE(model && cfg && keys_dev && psi0_dev && orb && spin, MCD_E_INVALID,
                "a required pointer is NULL");
    MCD_REQUIRE(n >= 1, MCD_E_INVALID, "empty basis");
    MCD_REQUIRE(n_sel >= 1 && n_sel <= 16, MCD_E_INVALID, "n_sel = %d outside 1..16", n_sel);
    MCD_REQUIRE(n_freq >= 0 && (n_freq == 0 || (omega && G_bar)), MCD_E_INVALID,
                "bad frequencies or G_bar");
    MCD_REQUIRE(cfg->w_t >= 1.0, MCD_E_INVALID, "the derivative needs w_t = 1 (no weight cut)");
    MCD_REQUIRE(cfg->max_blocks >= 1, MCD_E_INVALID, "max_blocks must be >= 1");
    MCD_REQUIRE(cfg->per_column == 0, MCD_E_INVALID, "the derivative uses block products");
    MCD_REQUIRE(cfg->precision == MCD_F64 || cfg->precision == MCD_F32, MCD_E_INVALID,
                "precision must be MCD_F64 or MCD_F32");
    MCD_REQUIRE(cg_tol > 0.0 && cg_max_iter >= 1, MCD_E_INVALID, "bad solve tolerance");
    HostModel hm;
    MCD_TRY(prepare_model(model, &hm));
    SelOps sel;
    memset(&sel, 0, sizeof(sel));
    sel.n = n_sel;
    for (int q = 0; q < n_sel; q++) {
        MCD_REQUIRE(orb[q] >= 0 && orb[q] < model->n_orb && (spin[q] == 0 || spin[q] == 1),
                    MCD_E_INVALID, "selection %d = (%d, %d) invalid", q, orb[q], spin[q]);
        sel.orb[q] = orb[q];
        sel.spin[q] = spin[q];
    }
    hipStream_t s = (hipStream_t)stream;
    if (keep) {   // the arguments must be those of the kept forward call
        bool same = keep->n == n && keep->n_sel == n_sel && keep->e0 == e0 &&
                    (int64_t)keep->omega.size() == n_freq &&
                    keep->cfg.max_blocks == cfg->max_blocks &&
                    keep->cfg.precision == cfg->precision && keep->cfg.dtol == cfg->dtol &&
                    keep->cfg.storage == cfg->storage && keep->cfg.reorth == cfg->reorth &&
                    keep->cfg.eta == cfg->eta && keep->cfg.g_tol == cfg->g_tol;
        for (int q = 0; same && q < n_sel; q++)
            same = keep->orb[q] == orb[q] && keep->spin[q] == spin[q];
        for (int f = 0; same && f < n_freq; f++) same = keep->omega[f] == omega[f];
        MCD_REQUIRE(same, MCD_E_INVALID,
                    "arguments differ from those of the kept forward call");
        MCD_REQUIRE(cfg->precision == MCD_F64 ? (bool)keep->kd : (bool)keep->kf, MCD_E_INVALID,
                    "kept run has another precision");
    }
    if (cfg->precision == MCD_F64)
        return band_green_vjp<double>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, cfg,
                                      G_bar, e0_bar, cg_tol, cg_max_iter, d_t, d_U, d_eps, info,
                                      ws, s, keep ? keep->kd.get() : nullptr);
    return band_green_vjp<float>(model, keys_dev, n, psi0_dev, e0, sel, n_freq, omega, cfg,
                                 G_bar, e0_bar, cg_tol, cg_max_iter, d_t, d_U, d_eps, info, ws, s,
                                 keep ? keep->kf.get() : nullptr);
}

extern "C" int mcd_band_green_vjp(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                                  const double *psi0_dev, double e0, int32_t n_sel,
                                  const int32_t *orb, const int32_t *spin, int32_t n_freq,
                                  const double *omega, const mcd_band_cfg *cfg,
                                  const double *G_bar, double e0_bar, double cg_tol,
                                  int32_t cg_max_iter, double *d_t, double *d_U, double *d_eps,
                                  mcd_solve_info *info, mcd_ws *ws, void *stream) {
    return band_vjp_entry(model, keys_dev, n, psi0_dev, e0, n_sel, orb, spin, n_freq, omega, cfg,
                          G_bar, e0_bar, cg_tol, cg_max_iter, d_t, d_U, d_eps, info, ws, stream,
                          nullptr);
}

extern "C" int mcd_band_green_vjp_keep(const mcd_model *model, const uint64_t *keys_dev,
                                       int64_t n, const double *psi0_dev, double e0,
                                       int32_t n_sel, const int32_t *orb, const int32_t *spin,
                                       int32_t n_freq, const double *omega,
                                       const mcd_band_cfg *cfg, const double *G_bar,
                                       double e0_bar, double cg_tol, int32_t cg_max_iter,
                                       double *d_t, double *d_U, double *d_eps,
                                       mcd_solve_info *info, mcd_ws *ws, void *stream,
                                       mcd_band_keep *keep) {
    MCD_REQUIRE(keep, MCD_E_INVALID, "keep is NULL");
    return band_vjp_entry(model, keys_dev, n, psi0_dev, e0, n_sel, orb, spin, n_freq, omega, cfg,
                          G_bar, e0_bar, cg_tol, cg_max_iter, d_t, d_U, d_eps, info, ws, stream,
                          keep);
}

extern "C" int mcd_batch_band_green(const mcd_model *const *models,
                                    const uint64_t *const *keys_dev, const int64_t *n,
                                    const double *const *psi0_dev, const double *e0,
                                    int32_t n_inst, int32_t n_sel, const int32_t *orb,
                                    const int32_t *spin, int32_t n_freq, const double *omega,
                                    const mcd_band_cfg *cfg, double *const *G_out,
                                    mcd_solve_info *info, mcd_ws *ws, void *stream) {
    MCD_REQUIRE(models && keys_dev && n && psi0_dev && e0 && orb && spin && cfg && G_out,
                MCD_E_INVALID, "a required pointer is NULL");
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "workspace is NULL");
    MCD_REQUIRE(n_inst >= 0, MCD_E_INVALID, "n_inst < 0");
    MCD_REQUIRE(n_sel >= 1 && n_sel <= 16, MCD_E_INVALID, "n_sel = %d outside 1..16", n_sel);
    MCD_REQUIRE(n_freq >= 0 && (n_freq == 0 || omega), MCD_E_INVALID, "bad frequencies");
    MCD_REQUIRE(cfg->w_t > 0.0 && cfg->w_t <= 1.0, MCD_E_INVALID, "w_t must be in (0, 1]");
    MCD_REQUIRE(cfg->max_blocks >= 1, MCD_E_INVALID, "max_blocks must be >= 1");
    MCD_REQUIRE(cfg->precision == MCD_F64 || cfg->precision == MCD_F32, MCD_E_INVALID,
                "precision must be MCD_F64 or MCD_F32");
    SelOps sel;
    memset(&sel, 0, sizeof(sel));
    sel.n = n_sel;
    for (int i = 0; i < n_inst; i++) {
        MCD_REQUIRE(models[i] && keys_dev[i] && psi0_dev[i] && G_out[i] && n[i] >= 1,
                    MCD_E_INVALID, "instance %d: missing input or empty basis", i);
        HostModel hm;
        MCD_TRY(prepare_model(models[i], &hm));
        for (int q = 0; q < n_sel; q++)
            MCD_REQUIRE(orb[q] >= 0 && orb[q] < models[i]->n_orb && (spin[q] == 0 || spin[q] == 1),
                        MCD_E_INVALID, "instance %d: selection %d = (%d, %d) invalid", i, q,
                        orb[q], spin[q]);
    }
    for (int q = 0; q < n_sel; q++) {
        sel.orb[q] = orb[q];
        sel.spin[q] = spin[q];
    }
    hipStream_t s = (hipStream_t)stream;
    auto go = [&](auto tag) -> int {
        using T = decltype(tag);
        std::vector<std::unique_ptr<Instance<T>>> own(n_inst);
        std::vector<Instance<T> *> inst(n_inst);
        for (int i = 0; i < n_inst; i++) {
            own[i].reset(new Instance<T>());
            Instance<T> &in = *own[i];
            in.model = models[i];
            in.keys = keys_dev[i];
            in.n = n[i];
            in.psi = psi0_dev[i];
            in.e0 = e0[i];
            in.G_out = G_out[i];
            inst[i] = own[i].get();
        }
        return band_green_multi<T>(inst, sel, n_freq, omega, cfg, ws, s, false, nullptr, false,
                                   info);
    };
    if (cfg->precision == MCD_F64) return go(double());
    return go(float());
}
