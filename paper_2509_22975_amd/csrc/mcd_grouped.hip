// Grouped entry order for the one-vector product y = H~ x (H~ = P H P on the
// basis, Eq. h_matrix_projected; elements from Eq. hubbard_model).
//
// With the basis sorted by (up string, down string), the rows sharing an up
// string u form a contiguous segment.  A down-spin hop keeps u, so its column
// lies in the row's own segment; an up-spin hop u -> u' = u ^ mask(bond) keeps
// the down string d, so for consecutive rows (u, d1), (u, d2), ... of one
// segment its columns (u', d1), (u', d2), ... are increasing positions inside
// segment u'.  In row-major order the lanes of one gather instruction take
// different hops of one row (up to ~30 different segments); here the entries
// of a row block are reordered so that they take the same hop u -> u' of
// consecutive rows, and the gathers of a wavefront fall on a few cache lines.
// Every entry keeps its row-major slot, so each row still adds its products
// in entry order and y is bit-identical to the row-major kernels.
//
// Layout, per row block [r0, r1) (<= kGroupedRows rows, <= kGroupedNnz
// nonzeros, found from the row pointers once):
//   entries: down hops sorted by column, then up-hop groups (source segment,
//   target segment) with columns ascending;
//   one 32-bit word per entry, bits 0-11 = row-major slot in the block;
//     down (bit 31 = 0): bits 12-26 column - r0 + 16384, 27-29 class, 30 sign
//     up   (bit 31 = 1): bits 12-23 column - group base, 24-30 group in block
//   group table (<= kGroupedMaxGroups per block), one 32-bit word per group:
//   base column (bits 0-27) | class << 28 | sign << 31 (an up hop's |t|
//   class and JW sign depend only on u and the bond, so they are the same
//   for every entry of a group).  Bits 27-30 of a down word and 28-31 of a
//   group word are both class | sign << 3: one signed-amplitude table of 16
//   entries serves both kinds.
// A basis whose segments are too short (many groups per block) or too long
// (offsets out of range) does not get the layout; the other kernels serve it.
//
// Kernels
//   k_g_rowmax     longest row
//   k_g_chunks     chunk k starts at the first row with rowptr >= k * step
//   k_g_pieces     rows of a chunk split into pieces of <= kGroupedRows
//   k_g_blocks     block row starts
//   k_g_heads      segment head flags (up string changes)
//   k_g_keys       sort key per entry: (block, up, source segment, column)
//   k_g_starts     group start flags in sorted order
//   k_g_entry_starts first entry of each block
//   k_g_goff       first group of each block; groups per block checked
//   k_g_tables     group table at each group start
//   k_g_words      entry words; ranges and group uniformity checked
//   k_spmv_grouped the product
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "mcd_internal.h"
#include "mcd_reduce.h"

namespace mcd {

namespace {

constexpr int BS = 256;

inline unsigned gridn(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + BS - 1) / BS); }

inline int bits_for(uint64_t v) {   // bits to hold values 0..v
    int b = 0;
    while (b < 64 && (v >> b) != 0) b++;
    return std::max(b, 1);
}

__global__ void k_g_rowmax(int64_t n, const int64_t *__restrict__ rowptr,
                           unsigned long long *__restrict__ out) {
    unsigned long long best = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        best = max(best, (unsigned long long)(rowptr[r + 1] - rowptr[r]));
    for (int off = 32; off > 0; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
    // one atomic per wavefront, and only where it can raise the maximum
    if ((threadIdx.x & 63) == 0 &&
        best > __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(out, best);
}

__global__ void k_g_chunks(int64_t n, int64_t nch, int64_t step, const int64_t *__restrict__ rowptr,
                           int64_t *__restrict__ cs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nch) return;
    if (k == nch) {
        cs[k] = n;
        return;
    }
    const int64_t target = k * step;
    int64_t lo = 0, hi = n;   // first r in [0, n] with rowptr[r] >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (rowptr[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    cs[k] = lo;
}

__global__ void k_g_pieces(int64_t nch, const int64_t *__restrict__ cs, int64_t *__restrict__ pc) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nch) return;
    if (k == nch) {
        pc[k] = 0;
        return;
    }
    const int64_t rows = cs[k + 1] - cs[k];
    pc[k] = (rows + kGroupedRows - 1) / kGroupedRows;
}

__global__ void k_g_blocks(int64_t n, int64_t nch, const int64_t *__restrict__ cs,
                           const int64_t *__restrict__ ps, int64_t nb, int64_t *__restrict__ gbs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nch) return;
    if (k == nch) {
        gbs[nb] = n;
        return;
    }
    const int64_t np = ps[k + 1] - ps[k];
    for (int64_t p = 0; p < np; p++) gbs[ps[k] + p] = cs[k] + p * kGroupedRows;
}

__global__ void k_g_heads(int64_t n, const uint64_t *__restrict__ keys, uint32_t *__restrict__ head) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    head[r] = (r == 0 || (keys[r] >> 32) != (keys[r - 1] >> 32)) ? 1u : 0u;
}

// One workgroup per row block; one thread per row, looping over its entries.
__global__ __launch_bounds__(BS) void k_g_keys(const int64_t *__restrict__ gbs,
                                               const int64_t *__restrict__ rowptr,
                                               const uint32_t *__restrict__ colw,
                                               const uint64_t *__restrict__ keys,
                                               const uint32_t *__restrict__ seg, uint32_t col_mask,
                                               int colbits, int segbits,
                                               uint64_t *__restrict__ skey,
                                               uint32_t *__restrict__ sval) {
    const int64_t b = blockIdx.x;
    const int64_t r = gbs[b] + threadIdx.x;
    if (r >= gbs[b + 1]) return;
    const uint32_t ur = (uint32_t)(keys[r] >> 32);
    const uint64_t bpart = (uint64_t)b << (1 + segbits + colbits);
    const uint64_t spart = ((uint64_t)1 << (segbits + colbits)) | ((uint64_t)seg[r] << colbits);
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; e++) {
        const uint32_t col = colw[e] & col_mask;
        const bool up = (uint32_t)(keys[col] >> 32) != ur;
        skey[e] = bpart | (up ? spart : 0ull) | (uint64_t)col;
        sval[e] = (uint32_t)e;
    }
}

__global__ void k_g_starts(int64_t nnz, const uint64_t *__restrict__ skey,
                           const uint64_t *__restrict__ keys, int colbits, int segbits,
                           uint32_t *__restrict__ flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const uint64_t k = skey[p];
    const uint64_t cmask = (colbits >= 64) ? ~0ull : ((1ull << colbits) - 1ull);
    const bool up = (k >> (segbits + colbits)) & 1ull;
    bool start = false;
    if (up) {
        if (p == 0) {
            start = true;
        } else {
            const uint64_t kp = skey[p - 1];
            start = (k >> colbits) != (kp >> colbits) ||
                    (keys[k & cmask] >> 32) != (keys[kp & cmask] >> 32);
        }
    }
    flag[p] = start ? 1u : 0u;
}

// gbe[b] = first entry of block b (its first row's row pointer).
__global__ void k_g_entry_starts(int64_t nb, const int64_t *__restrict__ gbs,
                                 const int64_t *__restrict__ rowptr, int64_t *__restrict__ gbe) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    gbe[b] = rowptr[gbs[b]];
}

// goff[b] = groups in the entries before block b (inclusive scan `gid`).
__global__ void k_g_goff(int64_t nb, const int64_t *__restrict__ gbs,
                         const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ gid,
                         int64_t *__restrict__ goff, int *__restrict__ bad) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    const int64_t e = rowptr[gbs[b]];
    goff[b] = e == 0 ? 0 : (int64_t)gid[e - 1];
    if (b < nb) {
        const int64_t e1 = rowptr[gbs[b + 1]];
        const int64_t g0 = e == 0 ? 0 : (int64_t)gid[e - 1];
        const int64_t g1 = e1 == 0 ? 0 : (int64_t)gid[e1 - 1];
        if (g1 - g0 > kGroupedMaxGroups) atomicOr(bad, 1);
    }
}

__global__ void k_g_tables(int64_t nnz, const uint32_t *__restrict__ sval,
                           const uint32_t *__restrict__ flag,
                           const uint32_t *__restrict__ gid, const uint32_t *__restrict__ colw,
                           uint32_t col_mask, int col_bits, uint32_t *__restrict__ gtab) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz || !flag[p]) return;
    const uint32_t w = colw[sval[p]];
    const uint32_t cls = (w & 0x7fffffffu) >> col_bits;
    // (a column past 28 bits or a class past 3 is caught by k_g_words)
    gtab[gid[p] - 1] = (w & col_mask & 0x0fffffffu) | ((uint32_t)(cls & 7u) << 28) |
                       ((w >> 31) << 31);
}

__global__ void k_g_words(int64_t nnz, const uint64_t *__restrict__ skey,
                          const uint32_t *__restrict__ sval, const uint32_t *__restrict__ gid,
                          const uint32_t *__restrict__ gtab, const int64_t *__restrict__ goff,
                          const int64_t *__restrict__ gbs, const int64_t *__restrict__ rowptr,
                          const uint32_t *__restrict__ colw, uint32_t col_mask, int col_bits,
                          int colbits, int segbits, uint32_t *__restrict__ gw,
                          int *__restrict__ bad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const uint64_t k = skey[p];
    const int64_t b = (int64_t)(k >> (1 + segbits + colbits));
    const bool up = (k >> (segbits + colbits)) & 1ull;
    const int64_t r0 = gbs[b];
    const int64_t slot = (int64_t)sval[p] - rowptr[r0];
    const uint32_t w = colw[sval[p]];
    const int64_t col = (int64_t)(w & col_mask);
    const uint32_t cls = (w & 0x7fffffffu) >> col_bits;
    const uint32_t sg = w >> 31;
    bool ok = slot >= 0 && slot < kGroupedNnz;
    uint32_t out = 0;
    if (!up) {
        const int64_t off = col - r0 + 16384;
        ok = ok && off >= 0 && off < 32768 && cls < 8u;
        out = (sg << 30) | (cls << 27) | ((uint32_t)(off & 32767) << 12) | (uint32_t)(slot & 4095);
    } else {
        const int64_t g = (int64_t)gid[p] - 1;
        const uint32_t t = gtab[g];
        const int64_t gl = g - goff[b];
        const int64_t off = col - (int64_t)(t & 0x0fffffffu);
        ok = ok && gl >= 0 && gl < kGroupedMaxGroups && off >= 0 && off < 4096 && cls < 8u &&
             col < (int64_t(1) << 28) && ((t >> 28) & 7u) == cls && (t >> 31) == sg;
        out = 0x80000000u | ((uint32_t)(gl & 127) << 24) | ((uint32_t)(off & 4095) << 12) |
              (uint32_t)(slot & 4095);
    }
    if (!ok) atomicOr(bad, 1);
    gw[p] = out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Decoding of an entry word v (layout above): the column it gathers and the
// index sc = class | sign << 3 of its signed amplitude.  ge = the block's
// group-table word of the group field of v (read for every word; a down
// word's bits 24-30 are its class, sign and high offset bits, so the read
// stays inside the 128-entry table and its value is not used); r0m = the
// block's first row - 16384, modulo 2^32.  Columns are < 2^28 (the layout is
// only built for such bases), so 32-bit arithmetic is exact and the two
// cases are selects, not branches.
__device__ __forceinline__ uint32_t g_decode(uint32_t v, uint32_t ge, uint32_t r0m, uint32_t &sc) {
    const bool up = (int32_t)v < 0;
    const uint32_t cu = (ge & 0x0fffffffu) + ((v >> 12) & 4095u);
    const uint32_t cd = r0m + ((v >> 12) & 32767u);
    sc = up ? (ge >> 28) : ((v >> 27) & 15u);
    return up ? cu : cd;
}

// x[col] for a column < 2^28 (a 32-bit byte offset from x).
template <typename T>
__device__ __forceinline__ T g_gather(const T *__restrict__ x, uint32_t col) {
    return *(const T *)((const char *)x + (size_t)(col * (uint32_t)sizeof(T)));
}

// Signed amplitudes amp[class | sign << 3] = +-|t_class| (into LDS by the
// first 16 threads).
template <typename T>
__device__ __forceinline__ void g_amp_table(const DevModel *__restrict__ m, T *amp) {
    const int t = threadIdx.x;
    if (t < 16) {
        const T a = (T)m->vtab[t & 7];
        amp[t] = (t & 8) ? -a : a;
    }
}

// The product.  A workgroup owns one row block: it loads the block's group
// table into LDS together with its rows' pointers, diagonal and x_r and its
// entry words (all unconditional loads on clamped addresses: the lanes past
// the block's last entry repeat it and so write the same value to the same
// slot), decodes the columns, issues the gathers, writes each signed product
// to the entry's row-major slot in LDS, and each row adds its run in entry
// order.  -(a x) and (-a) x are the same number, so y is bit-identical to
// the row-major kernels.
template <typename T, int NMAX>
__global__ __launch_bounds__(BS) void k_spmv_grouped(
    int64_t nblocks, const int64_t *__restrict__ gbs, const int64_t *__restrict__ gbe,
    const int64_t *__restrict__ goff, const uint32_t *__restrict__ gtab,
    const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ gw,
    const DevModel *__restrict__ m, const double *__restrict__ diag, const T *__restrict__ x,
    T *__restrict__ y, const double *__restrict__ sx_dev, int sx_mode,
    double *__restrict__ partials, int xcd_major) {
    constexpr int DEPTH = NMAX / BS;
    __shared__ T prod[NMAX];
    __shared__ T amp[16];
    __shared__ uint32_t gt[kGroupedMaxGroups];
    const int tid = threadIdx.x;
    int64_t blk = blockIdx.x;
    if (xcd_major) {
        const int64_t per = (nblocks + kNumXcd - 1) / kNumXcd;
        blk = (int64_t)(blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
    }
    if (blk >= nblocks) {   // padding workgroup of the XCD-major grid
        if (partials != nullptr && tid == 0) partials[blockIdx.x] = 0.0;
        return;
    }
    const int64_t r0 = gbs[blk], r1 = gbs[blk + 1];
    const int64_t g0 = goff[blk];
    const int ng = (int)(goff[blk + 1] - g0);
    const uint32_t gme = gtab[g0 + min(tid, ng)];   // table has one spare entry at the end
    const bool own = r0 + tid < r1;
    const int64_t r = min(r0 + (int64_t)tid, r1 - 1);
    const int64_t rs = rowptr[r], re = rowptr[r + 1];
    const double dr = diag[r];
    const T xr = x[r];
    const int64_t e0 = gbe[blk];
    const int cnt = (int)(gbe[blk + 1] - e0);
    uint32_t w[DEPTH];
#pragma unroll
    for (int j = 0; j < DEPTH; j++) w[j] = 0u;
    if (cnt > 0) {   // uniform over the workgroup
        const uint32_t *__restrict__ cw = gw + e0;
#pragma unroll
        for (int j = 0; j < DEPTH; j++)
            w[j] = *(const uint32_t *)((const char *)cw +
                                       (size_t)(4u * (uint32_t)min(tid + j * BS, cnt - 1)));
    }
    if (tid < ng && tid < kGroupedMaxGroups) gt[tid] = gme;
    g_amp_table<T>(m, amp);
    __syncthreads();
    if (cnt > 0) {
        const uint32_t r0m = (uint32_t)(r0 - 16384);
        T xv[DEPTH];
        uint32_t sc[DEPTH];
#pragma unroll
        for (int j = 0; j < DEPTH; j++)
            xv[j] = g_gather(x, g_decode(w[j], gt[(w[j] >> 24) & 127u], r0m, sc[j]));
#pragma unroll
        for (int j = 0; j < DEPTH; j++) prod[w[j] & 4095u] = amp[sc[j]] * xv[j];
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

template <typename T>
int grouped_one(const mcd_op *op, bool xcd, const T *x, T *y, const double *sx_dev, int sx_mode,
                double *partials, int64_t *grid, hipStream_t s) {
    MCD_REQUIRE(op->g_nblocks > 0, MCD_E_INVALID, "grouped layout not built for this operator");
    const int64_t nb = op->g_nblocks;
    const int64_t g = xcd ? kNumXcd * ((nb + kNumXcd - 1) / kNumXcd) : nb;
    MCD_REQUIRE(partials == nullptr || g <= op->max_partials, MCD_E_CAPACITY,
                "reduction scratch too small");
    hipLaunchKernelGGL((k_spmv_grouped<T, kGroupedNnz>), dim3((unsigned)g), dim3(BS), 0, s, nb,
                       op->d_gbs, op->d_gbe, op->d_goff, op->d_gtab, op->d_rowptr, op->d_gw,
                       op->d_model, op->d_diag, x, y, sx_dev, sx_mode, partials, xcd ? 1 : 0);
    MCD_HIP(hipGetLastError());
    *grid = g;
    return MCD_OK;
}

template int grouped_one<double>(const mcd_op *, bool, const double *, double *, const double *,
                                 int, double *, int64_t *, hipStream_t);
template int grouped_one<float>(const mcd_op *, bool, const float *, float *, const double *, int,
                                double *, int64_t *, hipStream_t);

// The takes and releases of build_grouped replayed on host bookkeeping with
// the largest sizes the layout can have (row blocks: at most two per chunk
// plus one per 256 rows; groups: at most one per nonzero), for the
// workspace-size query.
void grouped_plan(WsAlloc &w, int64_t n, int64_t nnz) {
    if (n == 0 || nnz <= 0 || nnz >= (int64_t(1) << 31)) return;
    hipStream_t s0 = (hipStream_t)0;
    std::vector<size_t> tmp;
    auto get = [&](size_t b) { tmp.push_back(w.alloc(std::max<size_t>(b, 8))); };
    size_t sb = 0, sb2 = 0, sb3 = 0, sb4 = 0;
    (void)hipcub::DeviceScan::InclusiveSum(nullptr, sb, (const uint32_t *)nullptr,
                                           (uint32_t *)nullptr, (int)n, s0);
    get(n * 4);
    get(n * 4);
    get(sb);
    get(8);
    const int64_t nch = nnz / (kGroupedNnz / 2) + 1;   // chunk step >= kGroupedNnz / 2
    get((nch + 1) * 8);
    get((nch + 1) * 8);
    get((nch + 1) * 8);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, sb2, (const int64_t *)nullptr,
                                           (int64_t *)nullptr, (int)(nch + 1), s0);
    get(sb2);
    const int64_t nb = 2 * nch + n / kGroupedRows + 2;
    w.alloc((nb + 1) * 8);   // d_gbs (kept)
    get(nnz * 8);
    get(nnz * 8);
    get(nnz * 4);
    get(nnz * 4);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sb3, (const uint64_t *)nullptr,
                                             (uint64_t *)nullptr, (const uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (int)nnz, 0, 64, s0);
    get(sb3);
    get(nnz * 4);
    get(nnz * 4);
    (void)hipcub::DeviceScan::InclusiveSum(nullptr, sb4, (const uint32_t *)nullptr,
                                           (uint32_t *)nullptr, (int)nnz, s0);
    get(sb4);
    get(sizeof(int));
    w.alloc((nb + 1) * 8);                                         // d_goff
    w.alloc((nb + 1) * 8);                                         // d_gbe
    w.alloc((size_t)(std::min<int64_t>(nnz, nb * kGroupedMaxGroups) + 1) * 4);   // d_gtab
    w.alloc(nnz * 4);                                              // d_gw
    for (size_t o : tmp) w.release(o);
}

// ---------------------------------------------------------------------------
// Build the layout from the packed CSR (rowptr, colw) and the sorted keys.
int build_grouped(mcd_op *op, hipStream_t s) {
    op->g_nblocks = 0;
    const int64_t n = op->n, nnz = op->nnz;
    if (n == 0 || nnz <= 0 || nnz >= (int64_t(1) << 31)) return MCD_OK;
    // a down-hop word holds a 3-bit amplitude class
    if (op->hm.dm.n_classes > 8) return MCD_OK;
    const Alloc &al = op->alloc;
    // Temporaries are released on every path.
    void *tmp[32] = {};
    int ntmp = 0;
    auto get = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t e = dmalloc(p, std::max<size_t>(bytes, 8), al);
        if (e == hipSuccess) tmp[ntmp++] = *p;
        return e;
    };
    auto release = [&]() {
        for (int i = 0; i < ntmp; i++) (void)dfree(tmp[i], al);
        ntmp = 0;
    };
    int rc = MCD_OK;
    int64_t *d_gbs = nullptr, *d_goff = nullptr, *d_gbe = nullptr;
    uint32_t *d_gtab = nullptr;
    uint32_t *d_gw = nullptr;
    auto fail_hip = [&](hipError_t e, const char *what) {
        (void)hipStreamSynchronize(s);   // queued work may still read the pieces
        release();
        for (void *p : {(void *)d_gbs, (void *)d_goff, (void *)d_gbe, (void *)d_gtab, (void *)d_gw})
            if (p) (void)dfree(p, al);
        if (e == hipErrorOutOfMemory) {   // no room in the workspace: no layout
            std::lock_guard<std::mutex> lock(al.ws->mu);
            al.ws->a.clear_need();
            return MCD_OK;
        }
        set_error("%s failed: %s", what, hipGetErrorString(e));
        return MCD_E_HIP;
    };
#define GK(expr)                                              \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return fail_hip(e_, #expr);     \
    } while (0)
    // Segments (rows sharing an up string): too short -> no layout.
    uint32_t *head = nullptr, *seg = nullptr;
    GK(get((void **)&head, n * sizeof(uint32_t)));
    GK(get((void **)&seg, n * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_g_heads, dim3(gridn(n)), dim3(BS), 0, s, n, op->d_keys, head);
    GK(hipGetLastError());
    size_t sb = 0;
    GK(hipcub::DeviceScan::InclusiveSum(nullptr, sb, head, seg, (int)n, s));
    void *scan_tmp = nullptr;
    GK(get(&scan_tmp, sb));
    GK(hipcub::DeviceScan::InclusiveSum(scan_tmp, sb, head, seg, (int)n, s));
    uint32_t nseg = 0;
    GK(hipMemcpyAsync(&nseg, seg + (n - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    unsigned long long *d_mx = nullptr;
    GK(get((void **)&d_mx, sizeof(unsigned long long)));
    GK(hipMemsetAsync(d_mx, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_g_rowmax, dim3(512), dim3(BS), 0, s, n, op->d_rowptr, d_mx);
    GK(hipGetLastError());
    unsigned long long maxrow = 0;
    GK(hipMemcpyAsync(&maxrow, d_mx, sizeof(maxrow), hipMemcpyDeviceToHost, s));
    GK(hipStreamSynchronize(s));
    if ((int64_t)nseg * 16 > n || maxrow >= (unsigned long long)(kGroupedNnz / 2) ||
        n >= (int64_t(1) << 28)) {   // columns must fit 28 bits
        release();
        return MCD_OK;
    }
    // Row blocks.
    const int64_t step = kGroupedNnz - (int64_t)maxrow;
    const int64_t nch = (nnz + step - 1) / step;
    int64_t *cs = nullptr, *pc = nullptr, *ps = nullptr;
    GK(get((void **)&cs, (nch + 1) * sizeof(int64_t)));
    GK(get((void **)&pc, (nch + 1) * sizeof(int64_t)));
    GK(get((void **)&ps, (nch + 1) * sizeof(int64_t)));
    hipLaunchKernelGGL(k_g_chunks, dim3(gridn(nch + 1)), dim3(BS), 0, s, n, nch, step,
                       op->d_rowptr, cs);
    hipLaunchKernelGGL(k_g_pieces, dim3(gridn(nch + 1)), dim3(BS), 0, s, nch, cs, pc);
    GK(hipGetLastError());
    size_t sb2 = 0;
    GK(hipcub::DeviceScan::ExclusiveSum(nullptr, sb2, pc, ps, (int)(nch + 1), s));
    void *scan2 = nullptr;
    GK(get(&scan2, sb2));
    GK(hipcub::DeviceScan::ExclusiveSum(scan2, sb2, pc, ps, (int)(nch + 1), s));
    int64_t nb = 0;
    GK(hipMemcpyAsync(&nb, ps + nch, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GK(hipStreamSynchronize(s));
    const int colbits = bits_for((uint64_t)n), segbits = bits_for((uint64_t)nseg);
    const int blkbits = bits_for((uint64_t)nb);
    if (nb <= 0 || blkbits + 1 + segbits + colbits > 64) {
        release();
        return MCD_OK;
    }
    GK(dmalloc((void **)&d_gbs, (nb + 1) * sizeof(int64_t), al));
    hipLaunchKernelGGL(k_g_blocks, dim3(gridn(nch + 1)), dim3(BS), 0, s, n, nch, cs, ps, nb, d_gbs);
    GK(hipGetLastError());
    // Sort the entries of every block by (up, source segment, column).
    uint64_t *k_in = nullptr, *k_out = nullptr;
    uint32_t *v_in = nullptr, *v_out = nullptr;
    GK(get((void **)&k_in, nnz * sizeof(uint64_t)));
    GK(get((void **)&k_out, nnz * sizeof(uint64_t)));
    GK(get((void **)&v_in, nnz * sizeof(uint32_t)));
    GK(get((void **)&v_out, nnz * sizeof(uint32_t)));
    const DevModel &dm = op->hm.dm;
    hipLaunchKernelGGL(k_g_keys, dim3((unsigned)nb), dim3(BS), 0, s, d_gbs, op->d_rowptr,
                       op->d_colw, op->d_keys, seg, dm.col_mask, colbits, segbits, k_in, v_in);
    GK(hipGetLastError());
    const int end_bit = blkbits + 1 + segbits + colbits;
    size_t sb3 = 0;
    GK(hipcub::DeviceRadixSort::SortPairs(nullptr, sb3, k_in, k_out, v_in, v_out, (int)nnz, 0,
                                          end_bit, s));
    void *sort_tmp = nullptr;
    GK(get(&sort_tmp, sb3));
    GK(hipcub::DeviceRadixSort::SortPairs(sort_tmp, sb3, k_in, k_out, v_in, v_out, (int)nnz, 0,
                                          end_bit, s));
    // Groups: start flags, ids (inclusive scan), per-block offsets, tables.
    uint32_t *flag = nullptr, *gid = nullptr;
    GK(get((void **)&flag, nnz * sizeof(uint32_t)));
    GK(get((void **)&gid, nnz * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_g_starts, dim3(gridn(nnz)), dim3(BS), 0, s, nnz, k_out, op->d_keys,
                       colbits, segbits, flag);
    GK(hipGetLastError());
    size_t sb4 = 0;
    GK(hipcub::DeviceScan::InclusiveSum(nullptr, sb4, flag, gid, (int)nnz, s));
    void *scan4 = nullptr;
    GK(get(&scan4, sb4));
    GK(hipcub::DeviceScan::InclusiveSum(scan4, sb4, flag, gid, (int)nnz, s));
    int *bad = nullptr;
    GK(get((void **)&bad, sizeof(int)));
    GK(hipMemsetAsync(bad, 0, sizeof(int), s));
    GK(dmalloc((void **)&d_goff, (nb + 1) * sizeof(int64_t), al));
    GK(dmalloc((void **)&d_gbe, (nb + 1) * sizeof(int64_t), al));
    hipLaunchKernelGGL(k_g_entry_starts, dim3(gridn(nb + 1)), dim3(BS), 0, s, nb, d_gbs,
                       op->d_rowptr, d_gbe);
    GK(hipGetLastError());
    hipLaunchKernelGGL(k_g_goff, dim3(gridn(nb + 1)), dim3(BS), 0, s, nb, d_gbs, op->d_rowptr, gid,
                       d_goff, bad);
    GK(hipGetLastError());
    uint32_t ngroups = 0;
    GK(hipMemcpyAsync(&ngroups, gid + (nnz - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    GK(hipStreamSynchronize(s));
    GK(dmalloc((void **)&d_gtab, ((int64_t)ngroups + 1) * sizeof(uint32_t), al));
    GK(hipMemsetAsync(d_gtab, 0, ((int64_t)ngroups + 1) * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_g_tables, dim3(gridn(nnz)), dim3(BS), 0, s, nnz, v_out, flag, gid,
                       op->d_colw, dm.col_mask, (int)dm.col_bits, d_gtab);
    GK(hipGetLastError());
    GK(dmalloc((void **)&d_gw, nnz * sizeof(uint32_t), al));
    hipLaunchKernelGGL(k_g_words, dim3(gridn(nnz)), dim3(BS), 0, s, nnz, k_out, v_out, gid, d_gtab,
                       d_goff, d_gbs, op->d_rowptr, op->d_colw, dm.col_mask, (int)dm.col_bits,
                       colbits, segbits, d_gw, bad);
    GK(hipGetLastError());
    int hbad = 0;
    GK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    GK(hipStreamSynchronize(s));
    release();
#undef GK
    if (hbad) {   // the basis does not fit the layout
        for (void *p : {(void *)d_gbs, (void *)d_goff, (void *)d_gbe, (void *)d_gtab, (void *)d_gw})
            (void)dfree(p, al);
        return rc;
    }
    op->g_nblocks = nb;
    op->g_ngroups = ngroups;
    op->d_gbs = d_gbs;
    op->d_goff = d_goff;
    op->d_gbe = d_gbe;
    op->d_gtab = d_gtab;
    op->d_gw = d_gw;
    op->device_bytes += 3 * (nb + 1) * 8 + (ngroups + 1) * 4 + nnz * 4;
    return rc;
}

}  // namespace mcd
