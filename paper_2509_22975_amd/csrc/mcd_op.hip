// The operator H~ = P H P on a truncated basis (Eq. h_matrix_projected):
// device index of the basis, diagonal, packed CSR build, and the applies.
//
// Kernels
//   k_validate      keys sorted, unique, within n_orb bits
//   k_diag          d_r = sum_i U_i n_iu n_id + sum_is eps_i n_is
//   k_hash_insert   open-addressing hash key -> row (load <= 1/4)
//   k_csr_count     kept hops per row (hop enumeration + lookup)
//   k_csr_fill      packed words: column | class << col_bits | sign << 31
//   k_block_max_all largest block nonzero count for every power-of-two block
//   k_spmv_grouped  (mcd_grouped.hip) one vector, grouped entry order
//   k_spmv_stream   one vector: a workgroup streams the nonzeros of a row
//                   block into LDS products, then each row sums its run
//   k_apply_group   nvec vectors (row-major): nvec lanes per row, each lane
//                   one column of the block; CSR or on-the-fly elements
//   k_block_csr(_v) nvec vectors from the CSR; _v gathers 16 bytes per lane
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>

#include "mcd_hash.h"
#include "mcd_internal.h"
#include "mcd_reduce.h"
#include "mcd_spmm.h"

namespace mcd {

__global__ void k_validate(int64_t n, const uint64_t *__restrict__ keys, int n_orb,
                           int *__restrict__ bad) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t k = keys[r];
    const uint64_t lim = (n_orb >= 32) ? 0xffffffffull : ((1ull << n_orb) - 1ull);
    bool ok = ((k >> 32) & ~lim) == 0 && ((k & 0xffffffffull) & ~lim) == 0;
    if (r + 1 < n) ok = ok && keys[r + 1] > k;
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_diag(int64_t n, const uint64_t *__restrict__ keys,
                       const DevModel *__restrict__ m, double *__restrict__ diag) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t k = keys[r];
    const uint32_t up = (uint32_t)(k >> 32), dn = (uint32_t)k;
    double d = 0.0;
    for (int i = 0; i < m->n_orb; i++) {
        const double nu = (double)((up >> i) & 1u), nd = (double)((dn >> i) & 1u);
        d += m->U[i] * (nu * nd);
        d += m->eps[i] * (nu + nd);
    }
    diag[r] = d;
}

__global__ void k_hash_insert(int64_t n, const uint64_t *__restrict__ keys, HashSlot *h,
                              uint64_t mask) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t key = keys[r];
    uint64_t p = mix64(key) & mask;
    for (;;) {
        unsigned long long prev = atomicCAS((unsigned long long *)&h[p].key,
                                            (unsigned long long)kEmpty, (unsigned long long)key);
        if (prev == kEmpty || prev == key) {
            h[p].val = r;
            return;
        }
        p = (p + 1) & mask;
    }
}

// Visit every kept hop of the state `key` in canonical order: the up-spin
// hops in bond order, then the down-spin hops in bond order.  Whether an up
// hop exists depends on the up string alone, so the rows of one up-string
// segment list their up hops first and alike: entry j of consecutive rows of
// a segment (in a full sector) is the same bond, whose images are
// consecutive rows of one target segment, and the row-parallel block
// products gather them together.  f(col, bond) is called for each image
// found in the basis; `neg` = element sign bit = JW parity XOR sign of t.
template <typename F>
__device__ __forceinline__ void for_each_hop(uint64_t key, const DevModel *__restrict__ m,
                                             const HashSlot *__restrict__ h, uint64_t hmask,
                                             F &&f) {
    const uint32_t up = (uint32_t)(key >> 32), dn = (uint32_t)key;
    const int nb = m->n_bonds;
    for (int b = 0; b < nb; b++) {
        const uint32_t mask = m->bonds[b].mask;
        if (__popc(up & mask) == 1) {
            const int64_t c = hash_find(h, hmask, key ^ ((uint64_t)mask << 32));
            if (c >= 0) f(c, b, (uint32_t)(__popc(up & m->bonds[b].between) & 1));
        }
    }
    for (int b = 0; b < nb; b++) {
        const uint32_t mask = m->bonds[b].mask;
        if (__popc(dn & mask) == 1) {
            const int64_t c = hash_find(h, hmask, key ^ (uint64_t)mask);
            if (c >= 0) f(c, b, (uint32_t)(__popc(dn & m->bonds[b].between) & 1));
        }
    }
}

// Candidate hops of a row, in for_each_hop's order (up-spin bonds, then
// down-spin bonds; a bond is a candidate when exactly one of its ends is
// occupied in that spin's string): at most 2 n_bonds, so up to 256 fit the
// four 64-bit words of a row's found mask.
constexpr int kFoundWords = 4;
inline int found_words(int n_bonds) {
    const int w = (2 * n_bonds + 63) / 64;
    return w <= kFoundWords ? std::max(w, 1) : 0;   // 0: no mask (every candidate probed twice)
}

// Kept hops per row; with `found` (nw words per row, word w of row r at
// found[w n + r]) also which candidates were found in the basis, so the fill
// probes only those.
__global__ void k_csr_count(int64_t n, const uint64_t *__restrict__ keys,
                            const DevModel *__restrict__ m, const HashSlot *__restrict__ h,
                            uint64_t hmask, int64_t *__restrict__ cnt,
                            uint64_t *__restrict__ found, int nw) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    if (r == n) {
        cnt[n] = 0;
        return;
    }
    if (found == nullptr) {
        int64_t c = 0;
        for_each_hop(keys[r], m, h, hmask, [&](int64_t, int, uint32_t) { c++; });
        cnt[r] = c;
        return;
    }
    const uint64_t key = keys[r];
    const uint32_t up = (uint32_t)(key >> 32), dn = (uint32_t)key;
    uint64_t f[kFoundWords] = {0, 0, 0, 0};
    int cand = 0;
    int64_t c = 0;
    const int nb = m->n_bonds;
    for (int spin = 0; spin < 2; spin++) {
        const uint32_t str = spin == 0 ? up : dn;
        for (int b = 0; b < nb; b++) {
            const uint32_t mask = m->bonds[b].mask;
            if (__popc(str & mask) != 1) continue;
            const uint64_t t = spin == 0 ? key ^ ((uint64_t)mask << 32) : key ^ (uint64_t)mask;
            if (hash_find(h, hmask, t) >= 0) {
                const uint64_t bit = 1ull << (cand & 63);
#pragma unroll
                for (int w = 0; w < kFoundWords; w++)
                    if ((cand >> 6) == w) f[w] |= bit;
                c++;
            }
            cand++;
        }
    }
    cnt[r] = c;
#pragma unroll
    for (int w = 0; w < kFoundWords; w++)
        if (w < nw) found[(int64_t)w * n + r] = f[w];
}

// Packed words of a row in for_each_hop's order; with `found`, only the
// candidates the count found are looked up (each lookup then hits).  The
// workgroup's rows own one contiguous range of words: when it fits
// kFillStage words, each thread writes its row's words into LDS and the
// workgroup then stores the range coalesced; otherwise straight to memory.
constexpr int kFillStage = 8192;
__global__ __launch_bounds__(256) void k_csr_fill(int64_t n, const uint64_t *__restrict__ keys,
                                                  const DevModel *__restrict__ m,
                                                  const HashSlot *__restrict__ h, uint64_t hmask,
                                                  const int64_t *__restrict__ rowptr,
                                                  uint32_t *__restrict__ colw,
                                                  const uint64_t *__restrict__ found, int nw) {
    __shared__ uint32_t stage[kFillStage];
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t r = r0 + threadIdx.x;
    const int64_t r1 = min(r0 + (int64_t)blockDim.x, n);   // r0 < n for every workgroup
    const int64_t w0 = rowptr[r0], w1 = rowptr[r1];
    const bool staged = w1 - w0 <= kFillStage;               // uniform over the workgroup
    const bool own = r < n;
    int64_t e = own ? rowptr[r] : 0;
    auto put = [&](uint32_t word) {
        if (staged)
            stage[e - w0] = word;
        else
            colw[e] = word;
        e++;
    };
    if (own) {
        if (found == nullptr) {
            for_each_hop(keys[r], m, h, hmask, [&](int64_t c, int b, uint32_t par) {
                const uint32_t neg = par ^ m->bonds[b].neg;
                put((uint32_t)c | (m->bonds[b].cls << m->col_bits) | (neg << 31));
            });
        } else {
            uint64_t f[kFoundWords] = {0, 0, 0, 0};
#pragma unroll
            for (int w = 0; w < kFoundWords; w++)
                if (w < nw) f[w] = found[(int64_t)w * n + r];
            const uint64_t key = keys[r];
            const uint32_t up = (uint32_t)(key >> 32), dn = (uint32_t)key;
            int cand = 0;
            const int nb = m->n_bonds;
            for (int spin = 0; spin < 2; spin++) {
                const uint32_t str = spin == 0 ? up : dn;
                for (int b = 0; b < nb; b++) {
                    const uint32_t mask = m->bonds[b].mask;
                    if (__popc(str & mask) != 1) continue;
                    uint64_t word = 0;
#pragma unroll
                    for (int w = 0; w < kFoundWords; w++)
                        if ((cand >> 6) == w) word = f[w];
                    if ((word >> (cand & 63)) & 1ull) {
                        const uint64_t t =
                            spin == 0 ? key ^ ((uint64_t)mask << 32) : key ^ (uint64_t)mask;
                        const int64_t c = hash_find(h, hmask, t);
                        if (c >= 0) {
                            const uint32_t par =
                                (uint32_t)(__popc(str & m->bonds[b].between) & 1);
                            const uint32_t neg = par ^ m->bonds[b].neg;
                            put((uint32_t)c | (m->bonds[b].cls << m->col_bits) | (neg << 31));
                        }
                    }
                    cand++;
                }
            }
        }
    }
    if (staged) {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < w1 - w0; i += blockDim.x) colw[w0 + i] = stage[i];
    }
}

// Largest nonzero count of a row block [b R, (b + 1) R) for every R = 2^k,
// k = 0..8, in one pass: out[k] (atomic max of wavefront maxima).
__global__ void k_block_max_all(int64_t n, const int64_t *__restrict__ rowptr,
                                unsigned long long *__restrict__ out) {
    unsigned long long best[9];
#pragma unroll
    for (int k = 0; k < 9; k++) best[k] = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const int64_t R = int64_t(1) << k;
            if ((r & (R - 1)) == 0)
                best[k] = max(best[k], (unsigned long long)(rowptr[min(r + R, n)] - rowptr[r]));
        }
    }
#pragma unroll
    for (int k = 0; k < 9; k++) {
        unsigned long long v = best[k];
        for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
        // the atomic only where it can raise the maximum: the wavefronts
        // would otherwise all queue on the same nine words
        if ((threadIdx.x & 63) == 0 &&
            v > __hip_atomic_load(&out[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&out[k], v);
    }
}

// ---------------------------------------------------------------------------
// One-vector CSR product.  A workgroup owns rows [r0, r0 + R) whose nonzeros
// (<= kStreamNnzMax) are contiguous.  The kernel is latency bound, so every
// thread first issues all its loads: its rows' pointers, diagonal and x_r,
// then up to DEPTH packed words (coalesced), then the DEPTH gathers of x;
// the signed products go to LDS and each row adds its run in entry order
// after d_r x_r.  Optional partial of sum_r (sx x_r) y_r per workgroup.
template <typename T, int BS, int NMAX>
__global__ __launch_bounds__(BS) void k_spmv_stream(
    int64_t n, int R, const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ colw,
    const DevModel *__restrict__ m, const double *__restrict__ diag, const T *__restrict__ x,
    T *__restrict__ y, const double *__restrict__ sx_dev, int sx_mode,
    double *__restrict__ partials, int64_t nblocks, int xcd_major) {
    constexpr int DEPTH = NMAX / BS;
    __shared__ T prod[NMAX];
    __shared__ T vtab[kMaxClasses];
    const int tid = threadIdx.x;
    // XCD-major mapping: workgroup b runs on XCD b % 8, so giving XCD k the
    // contiguous row blocks [k per, (k + 1) per) keeps each L2 on one slice of
    // the matrix (its gathers stay mostly in its own slice of x).
    int64_t blk = blockIdx.x;
    if (xcd_major) {
        const int64_t per = (nblocks + kNumXcd - 1) / kNumXcd;
        blk = (int64_t)(blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
    }
    if (blk >= nblocks) {   // padding workgroup of the XCD-major grid
        if (partials != nullptr && tid == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int64_t r0 = blk * R;
    const int64_t r1 = min(r0 + (int64_t)R, n);
    // Every load below is unconditional on a clamped, valid address (lanes
    // past the end are masked when the products are formed): no branches
    // around loads, so the compiler keeps them all in flight and waits by
    // count instead of draining the memory queue.
    const bool own = tid < R && r0 + tid < r1;
    const int64_t r = min(r0 + (int64_t)tid, r1 - 1);
    const int64_t rs = rowptr[r], re = rowptr[r + 1];
    const double dr = diag[r];
    const T xr = x[r];
    if (tid < kMaxClasses) vtab[tid] = (T)m->vtab[tid];
    const uint32_t cmask = m->col_mask, cbits = m->col_bits;
    const int64_t e0 = rowptr[r0];
    const int cnt = (int)(rowptr[r1] - e0);
    uint32_t w[DEPTH];
    T xv[DEPTH];
    if (cnt > 0) {   // uniform over the workgroup
        const uint32_t *__restrict__ cw = colw + e0;
#pragma unroll
        for (int j = 0; j < DEPTH; j++) w[j] = cw[min(tid + j * BS, cnt - 1)];
#pragma unroll
        for (int j = 0; j < DEPTH; j++) xv[j] = x[w[j] & cmask];
    }
    __syncthreads();
    if (cnt > 0) {
#pragma unroll
        for (int j = 0; j < DEPTH; j++) {
            const int e = tid + j * BS;
            if (e < cnt) {
                const T v = vtab[(w[j] & 0x7fffffffu) >> cbits];
                prod[e] = (w[j] >> 31) ? -(v * xv[j]) : v * xv[j];
            }
        }
    }
    __syncthreads();
    const double sx = scale_from(sx_dev, sx_mode);
    double dot = 0.0;
    if (own) {
        const int s0 = (int)(rs - e0), s1 = (int)(re - e0);
        T acc = (T)dr * xr;
#pragma unroll 4
        for (int k = s0; k < s1; k++) acc += prod[k];
        acc = acc * (T)sx;
        y[r] = acc;
        dot = (double)xr * sx * (double)acc;
    }
    if (partials != nullptr) store_partial<BS>(block_sum<BS>(dot), partials);
}

// ---------------------------------------------------------------------------
// One-vector CSR product, merge-path form.  The "path" of the matrix is the
// sequence (nonzeros of row 0, end of row 0, nonzeros of row 1, ...), a row
// end costing kMergeRowCost items; chunk c owns the items [c K, (c+1) K), so a
// chunk holds <= K nonzeros and ends < kMergeBS rows whatever the row lengths.
// Split points (rows ended, nonzeros consumed) are found once at build time.
// A persistent grid walks the chunks; while the products of chunk c are
// reduced, the packed words and row data of chunk c + grid are already in
// flight (their addresses do not depend on chunk c), which hides the load
// latency that bounds a one-chunk-per-workgroup kernel.  A row split across
// two chunks is finished by the first chunk that ends it; the other chunk's
// partial (its "carry") is added by k_merge_fixup, so every y_r is a fixed-
// order sum.  Row lengths must stay below K - kMergeRowCost (they are at
// most 2 n_bonds <= 1024 here).
__global__ void k_merge_splits(int64_t n, int64_t nch, const int64_t *__restrict__ rowptr,
                               int64_t *__restrict__ si, int64_t *__restrict__ sj) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nch) return;
    const int64_t nnz = rowptr[n];
    if (c == nch) {
        si[c] = n;
        sj[c] = nnz;
        return;
    }
    const int64_t d = c * (int64_t)kMergeK;
    // largest i in [0, n] with cost(i) = R i + rowptr[i] <= d
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)kMergeRowCost * mid + rowptr[mid] <= d)
            lo = mid;
        else
            hi = mid - 1;
    }
    si[c] = lo;
    sj[c] = (lo == n) ? nnz : min(d - (int64_t)kMergeRowCost * lo, rowptr[lo + 1]);
}

template <typename T>
struct MergeChunk {
    int64_t i0, i1, j0, j1;
    uint32_t w[kMergeDepth];
    int64_t rs, re;
    double d;
    T xr;
};

template <typename T>
__device__ __forceinline__ void merge_load(int64_t c, int64_t n, const int64_t *__restrict__ si,
                                           const int64_t *__restrict__ sj,
                                           const int64_t *__restrict__ rowptr,
                                           const uint32_t *__restrict__ colw,
                                           const double *__restrict__ diag,
                                           const T *__restrict__ x, MergeChunk<T> &q) {
    const int tid = threadIdx.x;
    q.i0 = si[c];
    q.i1 = si[c + 1];
    q.j0 = sj[c];
    q.j1 = sj[c + 1];
#pragma unroll
    for (int k = 0; k < kMergeDepth; k++) {
        const int64_t e = q.j0 + tid + k * kMergeBS;
        q.w[k] = (e < q.j1) ? colw[e] : 0u;
    }
    const int64_t r = q.i0 + tid;
    q.rs = 0;
    q.re = 0;
    q.d = 0.0;
    q.xr = (T)0;
    if (r <= q.i1 && r < n) {
        q.rs = rowptr[r];
        q.re = rowptr[r + 1];
    }
    if (r < q.i1) {
        q.d = diag[r];
        q.xr = x[r];
    }
}

template <typename T>
__global__ __launch_bounds__(kMergeBS) void k_spmv_merge(
    int64_t n, int64_t nch, const int64_t *__restrict__ si, const int64_t *__restrict__ sj,
    const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ colw,
    const DevModel *__restrict__ m, const double *__restrict__ diag, const T *__restrict__ x,
    T *__restrict__ y, double *__restrict__ carry, int64_t *__restrict__ carry_row,
    const double *__restrict__ sx_dev, int sx_mode, double *__restrict__ partials) {
    __shared__ T prod[kMergeK];
    __shared__ T vtab[kMaxClasses];
    const int tid = threadIdx.x;
    if (tid < kMaxClasses) vtab[tid] = (T)m->vtab[tid];
    const uint32_t cmask = m->col_mask, cbits = m->col_bits;
    const double sx = scale_from(sx_dev, sx_mode);
    double dot = 0.0;
    int64_t c = blockIdx.x;
    MergeChunk<T> cur, nxt;
    if (c < nch) merge_load(c, n, si, sj, rowptr, colw, diag, x, cur);
    __syncthreads();
    while (c < nch) {
        const int64_t cn = c + gridDim.x;
        T xv[kMergeDepth];
#pragma unroll
        for (int k = 0; k < kMergeDepth; k++) {
            const int64_t e = cur.j0 + tid + k * kMergeBS;
            xv[k] = (e < cur.j1) ? x[cur.w[k] & cmask] : (T)0;
        }
        if (cn < nch) merge_load(cn, n, si, sj, rowptr, colw, diag, x, nxt);
#pragma unroll
        for (int k = 0; k < kMergeDepth; k++) {
            const int64_t e = cur.j0 + tid + k * kMergeBS;
            if (e < cur.j1) {
                const uint32_t w = cur.w[k];
                const T v = vtab[(w & 0x7fffffffu) >> cbits];
                prod[e - cur.j0] = (w >> 31) ? -(v * xv[k]) : v * xv[k];
            }
        }
        __syncthreads();
        const int64_t r = cur.i0 + tid;
        if (r <= cur.i1) {
            if (r < n) {
                const int64_t a = max(cur.rs, cur.j0), b = min(cur.re, cur.j1);
                T acc = (T)0;
                for (int64_t e = a; e < b; e++) acc += prod[e - cur.j0];
                if (r < cur.i1) {
                    const T v = ((T)cur.d * cur.xr + acc) * (T)sx;
                    y[r] = v;
                    dot += (double)cur.xr * sx * (double)v;
                } else {
                    carry[c] = (double)(acc * (T)sx);
                    carry_row[c] = r;
                }
            } else {
                carry[c] = 0.0;
                carry_row[c] = n;
            }
        }
        __syncthreads();
        c = cn;
        cur = nxt;
    }
    if (partials != nullptr) store_partial<kMergeBS>(block_sum<kMergeBS>(dot), partials);
}

// y[carry_row[c]] += carry[c]; partial of sum (sx x_r) carry for the dot.
template <typename T>
__global__ __launch_bounds__(256) void k_merge_fixup(int64_t n, int64_t nch,
                                                     const double *__restrict__ carry,
                                                     const int64_t *__restrict__ carry_row,
                                                     const T *__restrict__ x, T *__restrict__ y,
                                                     const double *__restrict__ sx_dev,
                                                     int sx_mode, double *__restrict__ partials) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double dot = 0.0;
    if (c < nch) {
        const int64_t r = carry_row[c];
        if (r < n) {
            const double v = carry[c];
            y[r] = (T)((double)y[r] + v);
            dot = (double)x[r] * scale_from(sx_dev, sx_mode) * v;
        }
    }
    if (partials != nullptr) store_partial<256>(block_sum<256>(dot), partials);
}

// nvec lanes per row: lane k accumulates column k of the block.  CSR words
// are read once per group (same address for the group's lanes).  Each
// workgroup owns RT consecutive rows, walked RPB at a time, and the row tiles
// are dealt XCD-major (XCD k gets one contiguous slice of rows), so the
// gathered rows of X -- mostly inside the same up-string segment for
// down-spin hops -- are reused from that XCD's L2.
template <typename T, int NV, int BS, bool OTF, int CH = 16>
__global__ __launch_bounds__(BS) void k_apply_group(
    int64_t n, const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ colw,
    const DevModel *__restrict__ m, const uint64_t *__restrict__ keys,
    const HashSlot *__restrict__ h, uint64_t hmask, const double *__restrict__ diag,
    const T *__restrict__ x, T *__restrict__ y, int64_t ntiles, int rows_per_tile,
    const double *__restrict__ sx_dev = nullptr, int sx_mode = 0,
    double *__restrict__ partials = nullptr) {
    __shared__ T vtab[kMaxClasses];
    if (threadIdx.x < kMaxClasses) vtab[threadIdx.x] = (T)m->vtab[threadIdx.x];
    __syncthreads();
    const uint32_t cmask = m->col_mask, cbits = m->col_bits;
    constexpr int RPB = BS / NV;
    const int64_t per = (ntiles + kNumXcd - 1) / kNumXcd;
    const int64_t tile = (int64_t)(blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
    // optional scale sx and, for NV == 1, the partial of sum_r (sx x_r) y_r
    const double sx = scale_from(sx_dev, sx_mode);
    double dot = 0.0;
    if (tile >= ntiles) {
        if (partials != nullptr && threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int lane = threadIdx.x % NV;
    const int64_t rbeg = tile * rows_per_tile;
    const int64_t rend = min(rbeg + (int64_t)rows_per_tile, n);
    for (int64_t r = rbeg + threadIdx.x / NV; r < rend; r += RPB) {
        T acc = (T)diag[r] * x[r * NV + lane];
        if constexpr (!OTF) {
            // Chunks of CH nonzeros: the group loads the chunk's words with one
            // coalesced access (CH / NV words per lane), broadcasts word j with
            // a lane shuffle and issues all CH gathers before the first FMA, so
            // a row costs ~2 dependent memory round trips per chunk instead of
            // one per nonzero.  Accumulation stays in entry order.
            constexpr int WPL = (CH + NV - 1) / NV;
            const int64_t e1 = rowptr[r + 1];
            for (int64_t base = rowptr[r]; base < e1; base += CH) {
                uint32_t mw[WPL];
#pragma unroll
                for (int q = 0; q < WPL; q++) {
                    const int64_t e = base + q * NV + lane;
                    mw[q] = (q * NV + lane < CH && e < e1) ? colw[e] : 0u;
                }
                uint32_t wj[CH];
                T xv[CH];
#pragma unroll
                for (int j = 0; j < CH; j++) {
                    wj[j] = (uint32_t)__shfl((int)mw[j / NV], j % NV, NV);
                    xv[j] = (base + j < e1) ? x[(int64_t)(wj[j] & cmask) * NV + lane] : (T)0;
                }
#pragma unroll
                for (int j = 0; j < CH; j++) {
                    if (base + j < e1) {
                        const T v = vtab[(wj[j] & 0x7fffffffu) >> cbits];
                        acc += (wj[j] >> 31) ? -(v * xv[j]) : v * xv[j];
                    }
                }
            }
        } else {
            for_each_hop(keys[r], m, h, hmask, [&](int64_t c, int b, uint32_t par) {
                const T v = (T)m->bonds[b].t;
                const T xv = x[c * NV + lane];
                acc += par ? -(v * xv) : v * xv;
            });
        }
        if (sx_dev != nullptr) acc = acc * (T)sx;
        y[r * NV + lane] = acc;
        if (partials != nullptr) dot += (double)x[r * NV + lane] * sx * (double)acc;
    }
    if (partials != nullptr) store_partial<BS>(block_sum<BS>(dot), partials);
}

// Block product y = H~ X for NV vectors (row-major X[n][NV]) from the packed
// CSR, without the scaling / dot-product options of k_apply_group: NV lanes
// per row, the row's words loaded CH at a time (one coalesced access) and
// broadcast by lane shuffles, CH gathers of NV contiguous values in flight,
// sum in entry order.  CH follows the mean row length (short rows waste the
// masked slots of a long chunk).  XCD-major row tiles.
template <typename T, int NV, int CH>
__global__ __launch_bounds__(256) void k_block_csr(
    int64_t n, const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ colw,
    const DevModel *__restrict__ m, const double *__restrict__ diag, const T *__restrict__ x,
    T *__restrict__ y, int64_t ntiles, int rows_per_tile) {
    __shared__ T vtab[kMaxClasses];
    if (threadIdx.x < kMaxClasses) vtab[threadIdx.x] = (T)m->vtab[threadIdx.x];
    __syncthreads();
    const uint32_t cmask = m->col_mask, cbits = m->col_bits;
    constexpr int RPB = 256 / NV;
    constexpr int WPL = (CH + NV - 1) / NV;
    const int64_t per = (ntiles + kNumXcd - 1) / kNumXcd;
    const int64_t tile = (int64_t)(blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
    if (tile >= ntiles) return;
    const int lane = threadIdx.x % NV;
    const int64_t rbeg = tile * rows_per_tile;
    const int64_t rend = min(rbeg + (int64_t)rows_per_tile, n);
    for (int64_t r = rbeg + threadIdx.x / NV; r < rend; r += RPB) {
        T acc = (T)diag[r] * x[r * NV + lane];
        const int64_t e1 = rowptr[r + 1];
        for (int64_t base = rowptr[r]; base < e1; base += CH) {
            uint32_t mw[WPL];
#pragma unroll
            for (int q = 0; q < WPL; q++) {
                const int64_t e = base + q * NV + lane;
                mw[q] = (q * NV + lane < CH && e < e1) ? colw[e] : 0u;
            }
            uint32_t wj[CH];
            T xv[CH];
#pragma unroll
            for (int j = 0; j < CH; j++) {
                wj[j] = (uint32_t)__shfl((int)mw[j / NV], j % NV, NV);
                xv[j] = (base + j < e1) ? x[(int64_t)(wj[j] & cmask) * NV + lane] : (T)0;
            }
#pragma unroll
            for (int j = 0; j < CH; j++) {
                if (base + j < e1) {
                    const T v = vtab[(wj[j] & 0x7fffffffu) >> cbits];
                    acc += (wj[j] >> 31) ? -(v * xv[j]) : v * xv[j];
                }
            }
        }
        y[r * NV + lane] = acc;
    }
}

// k_block_csr with 16-byte gathers: L = NV / (16 / sizeof(T)) lanes per row,
// each lane 16 bytes of the gathered row (float4 / double2), so one gather
// instruction covers 4 / L times more rows; the same terms are added in the
// same order per column as in k_block_csr (bit-identical y).  X and Y
// 16-byte aligned.  XCD-major row tiles.
template <typename T, int NV, int CH, int WMAX>
__global__ __launch_bounds__(256) void k_block_csr_v(
    int64_t n, const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ colw,
    const DevModel *__restrict__ m, const double *__restrict__ diag, const T *__restrict__ x,
    T *__restrict__ y, int64_t ntiles, int rows_per_tile) {
    const int64_t per = (ntiles + kNumXcd - 1) / kNumXcd;
    const int64_t tile = (int64_t)(blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
    if (tile >= ntiles) return;   // whole workgroup, before any barrier
    const int64_t rbeg = tile * rows_per_tile;
    block_csr_v_tile<T, NV, CH, WMAX>(rowptr, colw, m, diag, x, y, rbeg,
                                      min(rbeg + (int64_t)rows_per_tile, n));
}

__global__ void k_conn_count(int64_t row0, int64_t row1, const uint64_t *__restrict__ keys,
                             const DevModel *__restrict__ m, const HashSlot *__restrict__ h,
                             uint64_t hmask, int64_t *__restrict__ cnt) {
    const int64_t r = row0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= row1) return;
    int64_t c = 0;
    for_each_hop(keys[r], m, h, hmask, [&](int64_t, int, uint32_t) { c++; });
    cnt[r - row0] = c;
}

__global__ void k_conn_fill(int64_t row0, int64_t row1, const uint64_t *__restrict__ keys,
                            const DevModel *__restrict__ m, const HashSlot *__restrict__ h,
                            uint64_t hmask, const int64_t *__restrict__ off,
                            int64_t *__restrict__ rows, int64_t *__restrict__ cols,
                            double *__restrict__ vals) {
    const int64_t r = row0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= row1) return;
    int64_t e = off[r - row0];
    for_each_hop(keys[r], m, h, hmask, [&](int64_t c, int b, uint32_t par) {
        rows[e] = r;
        cols[e] = c;
        vals[e] = par ? -m->bonds[b].t : m->bonds[b].t;
        e++;
    });
}

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Temporary bytes of the row-pointer scan (hipCUB) for n + 1 counts.
static size_t scan_tmp_bytes(int64_t n) {
    size_t b = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const int64_t *)nullptr,
                                           (int64_t *)nullptr, n + 1, (hipStream_t)0);
    return b;
}

static int64_t merge_chunks(int64_t n, int64_t nnz) {
    return std::max<int64_t>(1, (kMergeRowCost * n + nnz + kMergeK - 1) / kMergeK);
}

// CSR stage 1: row pointers (kept) from per-row counts of the kept hops.
// With `found` (op_create) the count also leaves each row's found-candidate
// mask in a workspace piece taken before the count's temporaries, for
// csr_fill, which releases it; without (the size query's probe) it counts
// only.
static int csr_count(mcd_op *op, hipStream_t s, uint64_t **found) {
    const int64_t n = op->n;
    int64_t *cnt = nullptr;
    void *tmp = nullptr;
    uint64_t *fm = nullptr;
    const int nw = found_words(op->hm.dm.n_bonds);
    MCD_HIP(dmalloc((void **)&op->d_rowptr, (n + 1) * sizeof(int64_t), op->alloc));
    op->device_bytes += (n + 1) * sizeof(int64_t);
    if (found && nw > 0) MCD_HIP(dmalloc((void **)&fm, (size_t)n * nw * sizeof(uint64_t), op->alloc));
    auto drop_mask = [&]() {
        if (fm) (void)dfree(fm, op->alloc);
        fm = nullptr;
    };
    {
        const hipError_t ec = dmalloc((void **)&cnt, (n + 1) * sizeof(int64_t), op->alloc);
        if (ec != hipSuccess) {
            drop_mask();
            MCD_HIP(ec);
        }
    }
    size_t tmp_bytes = scan_tmp_bytes(n);
    const hipError_t et = dmalloc(&tmp, tmp_bytes, op->alloc);
    if (et != hipSuccess) {
        (void)dfree(cnt, op->alloc);
        drop_mask();
        MCD_HIP(et);
    }
    hipLaunchKernelGGL(k_csr_count, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, n, op->d_keys,
                       op->d_model, op->d_hash, op->hash_mask, cnt, fm, nw);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, op->d_rowptr, n + 1, s);
    int64_t nnz = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nnz, op->d_rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)dfree(tmp, op->alloc);
    (void)dfree(cnt, op->alloc);
    if (e != hipSuccess) drop_mask();
    MCD_HIP(e);
    op->nnz = nnz;
    if (found) *found = fm;
    return MCD_OK;
}

// CSR stage 2: the packed words, the stream kernels' row blocks and the
// merge-path split points.
static int csr_fill(mcd_op *op, hipStream_t s, uint64_t *found) {
    const int64_t n = op->n, nnz = op->nnz;
    {
        const hipError_t ea = dmalloc((void **)&op->d_colw,
                                      std::max<int64_t>(nnz, 1) * sizeof(uint32_t), op->alloc);
        if (ea != hipSuccess) {
            if (found) (void)dfree(found, op->alloc);
            MCD_HIP(ea);
        }
    }
    op->device_bytes += nnz * sizeof(uint32_t);
    hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, n, op->d_keys,
                       op->d_model, op->d_hash, op->hash_mask, op->d_rowptr, op->d_colw, found,
                       found_words(op->hm.dm.n_bonds));
    if (found) (void)dfree(found, op->alloc);   // stream order: later work runs after the fill
    MCD_HIP(hipGetLastError());
    // Largest power-of-two row block whose nonzeros fit the LDS product buffer
    // (one choice per buffer size of the stream kernels), all sizes in one pass.
    unsigned long long *d_max = nullptr;
    MCD_HIP(dmalloc((void **)&d_max, 9 * sizeof(unsigned long long), op->alloc));
    unsigned long long mx[9] = {};
    hipError_t e = hipMemsetAsync(d_max, 0, 9 * sizeof(unsigned long long), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_block_max_all, dim3(512), dim3(256), 0, s, n, op->d_rowptr, d_max);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(mx, d_max, sizeof(mx), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)dfree(d_max, op->alloc);
    MCD_HIP(e);
    op->rows_per_block = 1;
    op->rows_per_block_s = 1;
    op->rows_per_block_l = 1;
    for (int k = 8; k >= 0; k--)
        if (mx[k] <= (unsigned long long)kStreamNnzMax) {
            op->rows_per_block = 1 << k;
            break;
        }
    for (int k = 8; k >= 0; k--)
        if (mx[k] <= (unsigned long long)kStreamNnzSmall) {
            op->rows_per_block_s = 1 << k;
            break;
        }
    for (int k = 8; k >= 0; k--)
        if (mx[k] <= (unsigned long long)kBlockWordsLarge) {
            op->rows_per_block_l = 1 << k;
            break;
        }
    // row-parallel products: words per chunk from the mean row length
    op->group_chunk = (nnz < 4 * n) ? 4 : (nnz < 10 * n) ? 8 : 16;
    // merge-path split points
    op->nchunks = merge_chunks(n, nnz);
    MCD_HIP(dmalloc((void **)&op->d_split_i, (op->nchunks + 1) * sizeof(int64_t), op->alloc));
    MCD_HIP(dmalloc((void **)&op->d_split_j, (op->nchunks + 1) * sizeof(int64_t), op->alloc));
    MCD_HIP(dmalloc((void **)&op->d_carry, op->nchunks * sizeof(double), op->alloc));
    MCD_HIP(dmalloc((void **)&op->d_carry_row, op->nchunks * sizeof(int64_t), op->alloc));
    MCD_HIP(poison_fp(op->d_carry, op->nchunks * sizeof(double), op->alloc, s));
    op->device_bytes += op->nchunks * 32;
    hipLaunchKernelGGL(k_merge_splits, dim3(grid_for(op->nchunks + 1, 256)), dim3(256), 0, s, n,
                       op->nchunks, op->d_rowptr, op->d_split_i, op->d_split_j);
    MCD_HIP(hipGetLastError());
    int dev = 0, cus = 256;
    MCD_HIP(hipGetDevice(&dev));
    MCD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    op->merge_grid = (int)std::min<int64_t>(op->nchunks, (int64_t)cus * 8);
    return MCD_OK;
}

// One-vector CSR product with the operator's selected kernel.
template <typename T>
static int csr_one(const mcd_op *op, const T *x, T *y, const double *sx_dev, int sx_mode,
                   double *dot_out, hipStream_t s) {
    const int64_t n = op->n;
    if (op->kernel == KERNEL_MERGE) {
        const int G = op->merge_grid;
        const int64_t nfix = (op->nchunks + 255) / 256;
        MCD_REQUIRE(!dot_out || G + nfix <= op->max_partials, MCD_E_CAPACITY,
                    "reduction scratch too small");
        hipLaunchKernelGGL((k_spmv_merge<T>), dim3(G), dim3(kMergeBS), 0, s, n, op->nchunks,
                           op->d_split_i, op->d_split_j, op->d_rowptr, op->d_colw, op->d_model,
                           op->d_diag, x, y, op->d_carry, op->d_carry_row, sx_dev, sx_mode,
                           dot_out ? op->d_partials : nullptr);
        hipLaunchKernelGGL((k_merge_fixup<T>), dim3((unsigned)nfix), dim3(256), 0, s, n,
                           op->nchunks, op->d_carry, op->d_carry_row, x, y, sx_dev, sx_mode,
                           dot_out ? op->d_partials + G : nullptr);
        MCD_HIP(hipGetLastError());
        if (dot_out) {
            hipLaunchKernelGGL((k_finalize_sum<1024>), dim3(1), dim3(1024), 0, s,
                               (int)(G + nfix), op->d_partials, dot_out);
            MCD_HIP(hipGetLastError());
        }
        return MCD_OK;
    }
    if (op->kernel == KERNEL_ROWCHUNK) {
        const int rpt = 1024;
        const int64_t ntiles = (n + rpt - 1) / rpt;
        const int64_t grid = kNumXcd * ((ntiles + kNumXcd - 1) / kNumXcd);
        MCD_REQUIRE(!dot_out || grid <= op->max_partials, MCD_E_CAPACITY,
                    "reduction scratch too small");
#define MCD_ROWCHUNK(C)                                                                      \
    hipLaunchKernelGGL((k_apply_group<T, 1, 256, false, C>), dim3((unsigned)grid), dim3(256), \
                       0, s, n, op->d_rowptr, op->d_colw, op->d_model, op->d_keys, op->d_hash, \
                       op->hash_mask, op->d_diag, x, y, ntiles, rpt, sx_dev, sx_mode,        \
                       dot_out ? op->d_partials : nullptr)
        if (op->group_chunk == 4)
            MCD_ROWCHUNK(4);
        else if (op->group_chunk == 8)
            MCD_ROWCHUNK(8);
        else
            MCD_ROWCHUNK(16);
#undef MCD_ROWCHUNK
        MCD_HIP(hipGetLastError());
        if (dot_out) {
            hipLaunchKernelGGL((k_finalize_sum<1024>), dim3(1), dim3(1024), 0, s, (int)grid,
                               op->d_partials, dot_out);
            MCD_HIP(hipGetLastError());
        }
        return MCD_OK;
    }
    if (op->kernel == KERNEL_GROUPED || op->kernel == KERNEL_GROUPED_XCD) {
        int64_t grid = 0;
        MCD_TRY(grouped_one<T>(op, op->kernel == KERNEL_GROUPED_XCD, x, y, sx_dev, sx_mode,
                               dot_out ? op->d_partials : nullptr, &grid, s));
        if (dot_out) {
            hipLaunchKernelGGL((k_finalize_sum<1024>), dim3(1), dim3(1024), 0, s, (int)grid,
                               op->d_partials, dot_out);
            MCD_HIP(hipGetLastError());
        }
        return MCD_OK;
    }
    const bool small = op->kernel == KERNEL_STREAM_S || op->kernel == KERNEL_STREAM_S_XCD;
    const int R = small ? op->rows_per_block_s : op->rows_per_block;
    const int64_t nb = (n + R - 1) / R;
    const bool xcd = op->kernel == KERNEL_STREAM_XCD || op->kernel == KERNEL_STREAM_S_XCD;
    const int64_t grid = xcd ? kNumXcd * ((nb + kNumXcd - 1) / kNumXcd) : nb;
    MCD_REQUIRE(!dot_out || grid <= op->max_partials, MCD_E_CAPACITY,
                "reduction scratch too small");
    if (small)
        hipLaunchKernelGGL((k_spmv_stream<T, 256, kStreamNnzSmall>), dim3((unsigned)grid),
                           dim3(256), 0, s, n, R, op->d_rowptr, op->d_colw, op->d_model,
                           op->d_diag, x, y, sx_dev, sx_mode, dot_out ? op->d_partials : nullptr,
                           nb, xcd ? 1 : 0);
    else
        hipLaunchKernelGGL((k_spmv_stream<T, 256, kStreamNnzMax>), dim3((unsigned)grid),
                           dim3(256), 0, s, n, R, op->d_rowptr, op->d_colw, op->d_model,
                           op->d_diag, x, y, sx_dev, sx_mode, dot_out ? op->d_partials : nullptr,
                           nb, xcd ? 1 : 0);
    MCD_HIP(hipGetLastError());
    if (dot_out) {
        hipLaunchKernelGGL((k_finalize_sum<1024>), dim3(1), dim3(1024), 0, s, (int)grid,
                           op->d_partials, dot_out);
        MCD_HIP(hipGetLastError());
    }
    return MCD_OK;
}

// Time every one-vector kernel on this matrix and keep the fastest (a
// per-operator autotune; a few applies of the diagonal as the vector).
static int tune_kernel(mcd_op *op, hipStream_t s) {
    if (op->n == 0) return MCD_OK;
    double *x = nullptr, *y = nullptr;
    MCD_HIP(dmalloc((void **)&x, op->n * sizeof(double), op->alloc));
    const hipError_t ey = dmalloc((void **)&y, op->n * sizeof(double), op->alloc);
    if (ey != hipSuccess) {
        (void)dfree(x, op->alloc);
        MCD_HIP(ey);
    }
    if (poison_fp(x, op->n * sizeof(double), op->alloc, s) != hipSuccess ||
        poison_fp(y, op->n * sizeof(double), op->alloc, s) != hipSuccess) {
        (void)hipStreamSynchronize(s);
        (void)dfree(x, op->alloc);
        (void)dfree(y, op->alloc);
        MCD_HIP(hipGetLastError());
        return MCD_E_HIP;
    }
    hipEvent_t a = nullptr, b = nullptr;
    auto done = [&](int rc) {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        (void)hipStreamSynchronize(s);   // the timed products read x and y
        (void)dfree(x, op->alloc);
        (void)dfree(y, op->alloc);
        return rc;
    };
#define TK(expr)                                           \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) {                            \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_)); \
            return done(MCD_E_HIP);                        \
        }                                                  \
    } while (0)
#define TT(expr)                  \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ < 0) return done(rc_); \
    } while (0)
    TK(hipMemcpyAsync(x, op->d_diag, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    TK(hipEventCreate(&a));
    TK(hipEventCreate(&b));
    double best = 1e300;
    int pick = KERNEL_STREAM;
    for (int k : {KERNEL_STREAM, KERNEL_STREAM_XCD, KERNEL_MERGE, KERNEL_ROWCHUNK,
                  KERNEL_STREAM_S, KERNEL_STREAM_S_XCD, KERNEL_GROUPED, KERNEL_GROUPED_XCD}) {
        op->tune_ms[k] = 0.0;
        if ((k == KERNEL_GROUPED || k == KERNEL_GROUPED_XCD) && op->g_nblocks == 0) continue;
        op->kernel = k;
        TT(csr_one<double>(op, x, y, nullptr, 0, nullptr, s));
        TK(hipEventRecord(a, s));
        const int reps = 5;
        for (int i = 0; i < reps; i++) TT(csr_one<double>(op, x, y, nullptr, 0, nullptr, s));
        TK(hipEventRecord(b, s));
        TK(hipEventSynchronize(b));
        float ms = 0.f;
        TK(hipEventElapsedTime(&ms, a, b));
        op->tune_ms[k] = ms / reps;
        if (ms < best) {
            best = ms;
            pick = k;
        }
    }
#undef TK
#undef TT
    // Between the plain and the XCD-major order of the same kernel, keep the
    // XCD-major one unless the plain one is clearly faster: it moves less
    // data over the fabric (each L2 serves its own slice of x).
    if (pick == KERNEL_STREAM && op->tune_ms[KERNEL_STREAM_XCD] <= 1.03 * op->tune_ms[KERNEL_STREAM])
        pick = KERNEL_STREAM_XCD;
    if (pick == KERNEL_STREAM_S &&
        op->tune_ms[KERNEL_STREAM_S_XCD] <= 1.03 * op->tune_ms[KERNEL_STREAM_S])
        pick = KERNEL_STREAM_S_XCD;
    if (pick == KERNEL_GROUPED &&
        op->tune_ms[KERNEL_GROUPED_XCD] <= 1.03 * op->tune_ms[KERNEL_GROUPED])
        pick = KERNEL_GROUPED_XCD;
    op->kernel = pick;
    return done(MCD_OK);
}

// Block CSR product with 16-byte gathers (k_block_csr_v), when a row of the
// block is a whole number of them; one-pass tiles (block_csr_v_tile), words
// per chunk from block_chunk.
template <typename T, int NV>
static void launch_block_v(const mcd_op *op, const T *x, T *y, hipStream_t s) {
    if constexpr (NV % Vec16<T>::n == 0) {
        constexpr int L = NV / Vec16<T>::n;
        const BlockTile bt = block_tile(L, op->rows_per_block, op->rows_per_block_l);
        const int rpt = bt.rows;
        const int ch = block_chunk(L, op->group_chunk);
        const int64_t n = op->n;
        const int64_t ntiles = (n + rpt - 1) / rpt;
        const unsigned grid = (unsigned)(kNumXcd * ((ntiles + kNumXcd - 1) / kNumXcd));
#define LBV(CH, WM)                                                                      \
    hipLaunchKernelGGL((k_block_csr_v<T, NV, CH, WM>), dim3(grid), dim3(256), 0, s, n,     \
                       op->d_rowptr, op->d_colw, op->d_model, op->d_diag, x, y, ntiles, rpt)
        if (!bt.large) {
            if (ch == 4) LBV(4, kStreamNnzMax);
            else if (ch == 8) LBV(8, kStreamNnzMax);
            else LBV(16, kStreamNnzMax);
        } else {
            if (ch == 4) LBV(4, kBlockWordsLarge);
            else if (ch == 8) LBV(8, kBlockWordsLarge);
            else LBV(16, kBlockWordsLarge);
        }
#undef LBV
    }
}

template <typename T>
static int launch_apply(const mcd_op *op, int nvec, const T *x, T *y, hipStream_t s) {
    const bool otf = op->storage == MCD_STORAGE_ON_THE_FLY;
    const int64_t n = op->n;
    if (n == 0) return MCD_OK;
    if (!otf && nvec == 1) return csr_one<T>(op, x, y, nullptr, 0, nullptr, s);
    const bool aligned16 = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15u) == 0;
    if (!otf && aligned16 && nvec % Vec16<T>::n == 0 && (nvec == 2 || nvec == 4 || nvec == 8 || nvec == 16)) {
        switch (nvec) {
            case 2: launch_block_v<T, 2>(op, x, y, s); break;
            case 4: launch_block_v<T, 4>(op, x, y, s); break;
            case 8: launch_block_v<T, 8>(op, x, y, s); break;
            case 16: launch_block_v<T, 16>(op, x, y, s); break;
        }
        MCD_HIP(hipGetLastError());
        return MCD_OK;
    }
    // row tile per workgroup: 4 passes of 256/NV rows (>= 64 rows)
#define MCD_GROUP(NV)                                                                          \
    case NV: {                                                                                 \
        const int rpt = std::max(64, 4 * (256 / NV));                                          \
        const int64_t ntiles = (n + rpt - 1) / rpt;                                            \
        const unsigned grid = (unsigned)(kNumXcd * ((ntiles + kNumXcd - 1) / kNumXcd));        \
        if (otf)                                                                               \
            hipLaunchKernelGGL((k_apply_group<T, NV, 256, true>), dim3(grid), dim3(256), 0, s, \
                               n, op->d_rowptr, op->d_colw, op->d_model, op->d_keys,           \
                               op->d_hash, op->hash_mask, op->d_diag, x, y, ntiles, rpt);      \
        else if (op->group_chunk == 4)                                                         \
            hipLaunchKernelGGL((k_block_csr<T, NV, 4>), dim3(grid), dim3(256), 0, s, n,        \
                               op->d_rowptr, op->d_colw, op->d_model, op->d_diag, x, y,        \
                               ntiles, rpt);                                                   \
        else if (op->group_chunk == 8)                                                         \
            hipLaunchKernelGGL((k_block_csr<T, NV, 8>), dim3(grid), dim3(256), 0, s, n,        \
                               op->d_rowptr, op->d_colw, op->d_model, op->d_diag, x, y,        \
                               ntiles, rpt);                                                   \
        else                                                                                   \
            hipLaunchKernelGGL((k_block_csr<T, NV, 16>), dim3(grid), dim3(256), 0, s, n,       \
                               op->d_rowptr, op->d_colw, op->d_model, op->d_diag, x, y,        \
                               ntiles, rpt);                                                   \
        break;                                                                                 \
    }
    switch (nvec) {
        MCD_GROUP(1)
        MCD_GROUP(2)
        MCD_GROUP(4)
        MCD_GROUP(8)
        MCD_GROUP(16)
        default:
            set_error("nvec = %d not in {1, 2, 4, 8, 16}", nvec);
            return MCD_E_INVALID;
    }
#undef MCD_GROUP
    MCD_HIP(hipGetLastError());
    return MCD_OK;
}

int apply_any(const mcd_op *op, int dtype, int nvec, const void *x, void *y, hipStream_t s) {
    if (dtype == MCD_F64) return launch_apply<double>(op, nvec, (const double *)x, (double *)y, s);
    if (dtype == MCD_F32) return launch_apply<float>(op, nvec, (const float *)x, (float *)y, s);
    set_error("dtype %d is neither MCD_F64 nor MCD_F32", dtype);
    return MCD_E_INVALID;
}

template <typename T>
int apply_fused(const mcd_op *op, const T *x, T *y, const double *sx_dev, int sx_mode,
                double *dot_out, hipStream_t s) {
    if (op->storage == MCD_STORAGE_CSR) return csr_one<T>(op, x, y, sx_dev, sx_mode, dot_out, s);
    // On-the-fly: product, then a separate fused scale + dot.
    MCD_TRY(launch_apply<T>(op, 1, x, y, s));
    if (sx_dev != nullptr || dot_out != nullptr)
        MCD_TRY(scale_dot<T>(op, y, x, sx_dev, sx_mode, dot_out, s));
    return MCD_OK;
}
template int apply_fused<double>(const mcd_op *, const double *, double *, const double *, int,
                                 double *, hipStream_t);
template int apply_fused<float>(const mcd_op *, const float *, float *, const double *, int,
                                double *, hipStream_t);

int apply_f64_fused(const mcd_op *op, const double *x, double *y, const double *sx_dev,
                    int sx_mode, double *dot_out, hipStream_t s) {
    return apply_fused<double>(op, x, y, sx_dev, sx_mode, dot_out, s);
}

static uint64_t hash_capacity(int64_t n) {
    const int64_t nn = std::max<int64_t>(n, 1);
    uint64_t cap = 16;
    while (cap < (uint64_t)(4 * nn)) cap <<= 1;   // load factor <= 1/4
    return cap;
}
static int64_t partials_capacity(int64_t n) { return std::max<int64_t>(n + 1024, 4096); }

// Stage "index": model, keys, diagonal, hash index (key -> row), reduction
// scratch; keys validated on request.
static int op_index(mcd_op *op, const uint64_t *keys_dev, int32_t validate, hipStream_t s) {
    const int64_t n = op->n, nn = std::max<int64_t>(n, 1);
    MCD_HIP(dmalloc((void **)&op->d_model, sizeof(DevModel), op->alloc));
    MCD_HIP(hipMemcpyAsync(op->d_model, &op->hm.dm, sizeof(DevModel), hipMemcpyHostToDevice, s));
    MCD_HIP(dmalloc((void **)&op->d_keys, nn * sizeof(uint64_t), op->alloc));
    if (n)
        MCD_HIP(hipMemcpyAsync(op->d_keys, keys_dev, n * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                               s));
    MCD_HIP(dmalloc((void **)&op->d_diag, nn * sizeof(double), op->alloc));
    MCD_HIP(poison_fp(op->d_diag, nn * sizeof(double), op->alloc, s));
    op->device_bytes = sizeof(DevModel) + nn * 16;
    if (validate && n) {
        int *bad = nullptr, hbad = 0;
        MCD_HIP(dmalloc((void **)&bad, sizeof(int), op->alloc));
        hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_validate, dim3(grid_for(n, 256)), dim3(256), 0, s, n, op->d_keys,
                               op->hm.dm.n_orb, bad);
            e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)dfree(bad, op->alloc);
        MCD_HIP(e);
        MCD_REQUIRE(!hbad, MCD_E_SECTOR, "keys are not sorted/unique or exceed n_orb bits");
    }
    if (n) {
        hipLaunchKernelGGL(k_diag, dim3(grid_for(n, 256)), dim3(256), 0, s, n, op->d_keys,
                           op->d_model, op->d_diag);
        MCD_HIP(hipGetLastError());
    }
    const uint64_t cap = hash_capacity(n);
    op->hash_mask = cap - 1;
    MCD_HIP(dmalloc((void **)&op->d_hash, cap * sizeof(HashSlot), op->alloc));
    MCD_HIP(hipMemsetAsync(op->d_hash, 0xff, cap * sizeof(HashSlot), s));
    op->device_bytes += cap * sizeof(HashSlot);
    if (n) {
        hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(n, 256)), dim3(256), 0, s, n, op->d_keys,
                           op->d_hash, op->hash_mask);
        MCD_HIP(hipGetLastError());
    }
    op->max_partials = partials_capacity(n);
    MCD_HIP(dmalloc((void **)&op->d_partials, op->max_partials * sizeof(double), op->alloc));
    MCD_HIP(dmalloc((void **)&op->d_counter, 8 * sizeof(unsigned int), op->alloc));
    MCD_HIP(hipMemsetAsync(op->d_counter, 0, 8 * sizeof(unsigned int), s));
    MCD_HIP(dmalloc((void **)&op->d_scalars, 64 * sizeof(double), op->alloc));
    MCD_HIP(poison_fp(op->d_partials, op->max_partials * sizeof(double), op->alloc, s));
    MCD_HIP(poison_fp(op->d_scalars, 64 * sizeof(double), op->alloc, s));
    op->device_bytes += op->max_partials * sizeof(double);
    return MCD_OK;
}

// The CSR pieces of stage "fill" (for the fallback of AUTO to on-the-fly).
static void release_csr(mcd_op *op) {
    for (void **p : {(void **)&op->d_rowptr, (void **)&op->d_colw, (void **)&op->d_split_i,
                     (void **)&op->d_split_j, (void **)&op->d_carry, (void **)&op->d_carry_row}) {
        (void)dfree(*p, op->alloc);
        *p = nullptr;
    }
}

// Bytes op_create takes from an empty workspace: its sequence of takes and
// releases replayed on the host bookkeeping (stage 1: index only, 2: up to
// the nonzero count, 3: everything but the optional grouped layout, 4: with
// a grouped layout of the largest possible size).
size_t op_plan(int64_t n, bool csr, int64_t nnz, bool tune, bool validate, int stages,
               int n_bonds) {
    WsAlloc w(size_t(1) << 62);
    const int64_t nn = std::max<int64_t>(n, 1);
    std::vector<size_t> keep;
    auto take = [&](size_t b) { size_t o = w.alloc(b); keep.push_back(o); return o; };
    auto temp = [&](size_t b) { return w.alloc(b); };
    take(sizeof(DevModel));
    take(nn * 8);
    take(nn * 8);
    if (validate && n) w.release(temp(sizeof(int)));
    take(hash_capacity(n) * sizeof(HashSlot));
    take(partials_capacity(n) * 8);
    take(8 * sizeof(unsigned int));
    take(64 * 8);
    // the found-candidate mask is taken by op_create's count (stage 3 plans),
    // not by the size query's probe (stage 2 alone)
    const int nw = found_words(n_bonds);
    const bool mask = stages >= 3 && csr && nw > 0 && n > 0;
    size_t fm = 0;
    if (stages >= 2 && csr) {
        take((n + 1) * 8);
        if (mask) fm = temp((size_t)n * nw * 8);
        const size_t c = temp((n + 1) * 8), t = temp(scan_tmp_bytes(n));
        w.release(t);
        w.release(c);
    }
    if (stages >= 3 && csr) {
        take(std::max<int64_t>(nnz, 1) * 4);
        if (mask) w.release(fm);
        w.release(temp(9 * 8));
        const int64_t nch = merge_chunks(n, nnz);
        take((nch + 1) * 8);
        take((nch + 1) * 8);
        take(nch * 8);
        take(nch * 8);
        if (stages >= 4 && tune) grouped_plan(w, n, nnz);
        if (tune && n) {
            const size_t x = temp(n * 8), y = temp(n * 8);
            w.release(x);
            w.release(y);
        }
    }
    return w.extent();
}

// Operator construction; `tune` times the one-vector kernels on the matrix
// (operators that only ever see block products skip it and keep the
// XCD-major stream kernel for the rare one-vector product) and builds the
// grouped layout when the workspace has room for it.
int op_create(const mcd_model *model, const uint64_t *keys_dev, int64_t n, int32_t storage,
              int32_t validate, bool tune, mcd_ws *ws, void *stream, mcd_op **out) {
    MCD_REQUIRE(out != nullptr, MCD_E_INVALID, "out is NULL");
    *out = nullptr;
    MCD_REQUIRE(n >= 0 && (n == 0 || keys_dev != nullptr), MCD_E_INVALID, "bad keys/n");
    MCD_REQUIRE(storage >= MCD_STORAGE_AUTO && storage <= MCD_STORAGE_CSR, MCD_E_INVALID,
                "storage %d unknown", storage);
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    const double t0 = now_ms();
    mcd_op *op = new mcd_op();
    memset(op, 0, sizeof(*op));
    op->alloc.ws = ws;
    auto fail = [&](int rc) {
        mcd_op_destroy(op);
        return rc;
    };
    int rc = prepare_model(model, &op->hm);
    if (rc < 0) return fail(rc);
    if (hipGetDevice(&op->device) != hipSuccess) return fail(MCD_E_HIP);
    op->n = n;
    op->nnz = -1;
    rc = op_index(op, keys_dev, validate, s);
    if (rc < 0) return fail(rc);
    // Storage choice: AUTO takes the CSR when the format fits and the
    // workspace holds it, else recomputes the elements at every product.
    const bool fmt_ok = n <= (int64_t(1) << op->hm.dm.col_bits) && op->hm.ok_classes;
    int st = storage;
    if (st == MCD_STORAGE_CSR && !fmt_ok) {
        set_error("packed CSR needs n <= 2^%u (%d amplitude classes) and <= 32 distinct |t| "
                  "(n = %lld)", op->hm.dm.col_bits, op->hm.dm.n_classes, (long long)n);
        return fail(MCD_E_CAPACITY);
    }
    if (st == MCD_STORAGE_AUTO) st = fmt_ok ? MCD_STORAGE_CSR : MCD_STORAGE_ON_THE_FLY;
    op->rows_per_block = 256;
    op->rows_per_block_s = 256;
    op->rows_per_block_l = 256;
    op->group_chunk = 16;
    op->kernel = KERNEL_STREAM_XCD;
    if (st == MCD_STORAGE_CSR) {
        uint64_t *found = nullptr;
        rc = csr_count(op, s, &found);
        if (rc >= 0) rc = csr_fill(op, s, found);
        if (rc == MCD_E_WORKSPACE && storage == MCD_STORAGE_AUTO) {
            // no room for the CSR: elements on the fly instead
            (void)hipStreamSynchronize(s);
            release_csr(op);
            op->nnz = -1;
            op->device_bytes = sizeof(DevModel) + std::max<int64_t>(n, 1) * 16 +
                               hash_capacity(n) * sizeof(HashSlot) + op->max_partials * 8;
            {
                std::lock_guard<std::mutex> lock(ws->mu);
                ws->a.clear_need();
            }
            st = MCD_STORAGE_ON_THE_FLY;
            rc = MCD_OK;
        }
        if (rc < 0) return fail(rc);
    }
    op->storage = st;
    if (st == MCD_STORAGE_CSR && tune) {
        rc = build_grouped(op, s);   // skipped when the workspace has no room
        if (rc >= 0) rc = tune_kernel(op, s);
        if (rc < 0) return fail(rc);
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MCD_E_HIP);
    op->build_ms = now_ms() - t0;
    *out = op;
    return MCD_OK;
}

}  // namespace mcd

using namespace mcd;

extern "C" int mcd_op_create(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                             int32_t storage, int32_t validate, mcd_ws *ws, void *stream,
                             mcd_op **out) {
    return op_create(model, keys_dev, n, storage, validate, true, ws, stream, out);
}

extern "C" int mcd_op_workspace_size(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                                     int32_t storage, mcd_ws *ws, void *stream, size_t *bytes,
                                     size_t *bytes_grouped) {
    MCD_REQUIRE(bytes != nullptr, MCD_E_INVALID, "bytes is NULL");
    MCD_REQUIRE(n >= 0 && (n == 0 || keys_dev != nullptr), MCD_E_INVALID, "bad keys/n");
    MCD_REQUIRE(storage >= MCD_STORAGE_AUTO && storage <= MCD_STORAGE_CSR, MCD_E_INVALID,
                "storage %d unknown", storage);
    HostModel hm;
    MCD_TRY(prepare_model(model, &hm));
    const bool fmt_ok = n <= (int64_t(1) << hm.dm.col_bits) && hm.ok_classes;
    MCD_REQUIRE(storage != MCD_STORAGE_CSR || fmt_ok, MCD_E_CAPACITY,
                "packed CSR needs n <= 2^%u and <= 32 distinct |t|", hm.dm.col_bits);
    if (storage == MCD_STORAGE_ON_THE_FLY || !fmt_ok) {
        *bytes = op_plan(n, false, 0, false, true, 3, hm.dm.n_bonds);
        if (bytes_grouped) *bytes_grouped = *bytes;
        return MCD_OK;
    }
    // The CSR size needs the nonzero count: index and count in the caller's
    // probe workspace (its size is the answer when ws is NULL or too small).
    const size_t probe = op_plan(n, true, 0, false, true, 2, hm.dm.n_bonds);
    if (ws == nullptr || ws->a.size() < probe) {
        *bytes = probe;
        if (bytes_grouped) *bytes_grouped = probe;
        set_error("counting the nonzeros needs a probe workspace of %zu bytes", probe);
        return MCD_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    mcd_op *op = new mcd_op();
    memset(op, 0, sizeof(*op));
    op->alloc.ws = ws;
    op->hm = hm;
    op->n = n;
    int rc = hipGetDevice(&op->device) == hipSuccess ? MCD_OK : MCD_E_HIP;
    if (rc >= 0) rc = op_index(op, keys_dev, 0, s);
    if (rc >= 0) rc = csr_count(op, s, nullptr);
    const int64_t nnz = op->nnz;
    (void)hipStreamSynchronize(s);
    mcd_op_destroy(op);
    MCD_TRY(rc);
    *bytes = op_plan(n, true, nnz, true, true, 3, hm.dm.n_bonds);
    if (bytes_grouped)
        *bytes_grouped = std::max(*bytes, op_plan(n, true, nnz, true, true, 4, hm.dm.n_bonds));
    return MCD_OK;
}

extern "C" void mcd_op_destroy(mcd_op *op) {
    if (!op) return;
    // Pieces go back to the caller's workspace; work still queued on the
    // caller's stream that reads them runs before any later use of the
    // workspace on that stream.
    for (void *p : {(void *)op->d_model, (void *)op->d_keys, (void *)op->d_diag,
                    (void *)op->d_hash, (void *)op->d_rowptr, (void *)op->d_colw,
                    (void *)op->d_partials, (void *)op->d_counter, (void *)op->d_scalars,
                    (void *)op->d_split_i, (void *)op->d_split_j, (void *)op->d_carry,
                    (void *)op->d_carry_row, (void *)op->d_gbs, (void *)op->d_goff,
                    (void *)op->d_gbe, (void *)op->d_gtab, (void *)op->d_gw})
        if (p) (void)dfree(p, op->alloc);
    delete op;
}

extern "C" int mcd_op_info(const mcd_op *op, mcd_op_info_t *info) {
    MCD_REQUIRE(op && info, MCD_E_INVALID, "op or info is NULL");
    info->n = op->n;
    info->nnz = op->storage == MCD_STORAGE_CSR ? op->nnz : -1;
    info->storage = op->storage;
    info->n_classes = op->hm.dm.n_classes;
    info->rows_per_block = op->rows_per_block;
    info->rows_per_block_l = op->rows_per_block_l;
    info->kernel = op->kernel;
    info->device_bytes = op->device_bytes;
    info->build_ms = op->build_ms;
    info->grouped_blocks = op->g_nblocks;
    info->grouped_groups = op->g_nblocks > 0 ? op->g_ngroups : 0;
    info->reserved = 0;
    return MCD_OK;
}

extern "C" int mcd_op_set_kernel(mcd_op *op, int32_t kernel) {
    MCD_REQUIRE(op != nullptr, MCD_E_INVALID, "op is NULL");
    MCD_REQUIRE(op->storage == MCD_STORAGE_CSR, MCD_E_INVALID, "operator has no CSR");
    MCD_REQUIRE(kernel >= KERNEL_STREAM && kernel <= KERNEL_LAST, MCD_E_INVALID,
                "kernel %d unknown", kernel);
    MCD_REQUIRE(op->g_nblocks > 0 || (kernel != KERNEL_GROUPED && kernel != KERNEL_GROUPED_XCD),
                MCD_E_INVALID, "the grouped layout was not built for this operator (kernel %d)",
                kernel);
    op->kernel = kernel;
    return MCD_OK;
}

extern "C" int mcd_hamiltonian_apply(const mcd_op *op, int32_t dtype, int32_t nvec,
                                     const void *x_dev, void *y_dev, void *stream) {
    MCD_REQUIRE(op != nullptr, MCD_E_INVALID, "op is NULL");
    MCD_REQUIRE(op->n == 0 || (x_dev && y_dev), MCD_E_INVALID, "x or y is NULL");
    MCD_REQUIRE(x_dev != y_dev || op->n == 0, MCD_E_INVALID, "x and y must not alias");
    return apply_any(op, dtype, nvec, x_dev, y_dev, (hipStream_t)stream);
}

extern "C" int mcd_hamiltonian_diagonal(const mcd_op *op, double *diag_dev, void *stream) {
    MCD_REQUIRE(op && (diag_dev || op->n == 0), MCD_E_INVALID, "op or diag is NULL");
    if (op->n)
        MCD_HIP(hipMemcpyAsync(diag_dev, op->d_diag, op->n * sizeof(double),
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MCD_OK;
}

extern "C" int mcd_hamiltonian_connectivity(const mcd_op *op, int64_t row0, int64_t row1,
                                            int64_t *rows_dev, int64_t *cols_dev,
                                            double *vals_dev, int64_t cap, int64_t *count_out,
                                            mcd_ws *ws, void *stream) {
    MCD_REQUIRE(op && count_out, MCD_E_INVALID, "op or count_out is NULL");
    MCD_REQUIRE(0 <= row0 && row0 <= row1 && row1 <= op->n, MCD_E_INVALID,
                "row range [%lld, %lld) outside [0, %lld)", (long long)row0, (long long)row1,
                (long long)op->n);
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = row1 - row0;
    *count_out = 0;
    if (m == 0) return MCD_OK;
    const Alloc al{ws};
    int64_t *cnt = nullptr;
    MCD_HIP(dmalloc((void **)&cnt, m * sizeof(int64_t), al));
    hipLaunchKernelGGL(k_conn_count, dim3(grid_for(m, 256)), dim3(256), 0, s, row0, row1,
                       op->d_keys, op->d_model, op->d_hash, op->hash_mask, cnt);
    std::vector<int64_t> h(m);
    MCD_HIP(hipMemcpyAsync(h.data(), cnt, m * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MCD_HIP(hipStreamSynchronize(s));
    int64_t tot = 0;
    for (int64_t i = 0; i < m; i++) {
        const int64_t c = h[i];
        h[i] = tot;
        tot += c;
    }
    *count_out = tot;
    if (tot > cap) {
        (void)dfree(cnt, al);
        set_error("connectivity needs %lld entries, cap is %lld", (long long)tot, (long long)cap);
        return MCD_E_CAPACITY;
    }
    if (tot > 0 && !(rows_dev && cols_dev && vals_dev)) {
        (void)dfree(cnt, al);
        set_error("outputs NULL");
        return MCD_E_INVALID;
    }
    MCD_HIP(hipMemcpyAsync(cnt, h.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_conn_fill, dim3(grid_for(m, 256)), dim3(256), 0, s, row0, row1,
                       op->d_keys, op->d_model, op->d_hash, op->hash_mask, cnt, rows_dev,
                       cols_dev, vals_dev);
    MCD_HIP(hipGetLastError());
    MCD_HIP(hipStreamSynchronize(s));
    MCD_HIP(dfree(cnt, al));
    return MCD_OK;
}
