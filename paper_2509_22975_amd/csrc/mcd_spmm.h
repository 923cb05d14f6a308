// Block product of the packed CSR with 16-byte gathers, as a device
// function over one tile of rows, shared by the one-operator kernel
// (mcd_op.hip) and the kernel that serves many band runs in one launch
// (mcd_band.hip), and the rule that sizes its tiles.
#pragma once

#include <hip/hip_runtime.h>

#include "mcd_internal.h"

namespace mcd {

// Vector types of one 16-byte gather.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};

// Words per chunk of the block product with L lanes per row (measured on
// gfx950, C2 basis, 8 and 16 vectors): at most 8 gathers in flight per lane
// at L >= 4 (ch: words per chunk from the mean row length).  It does not
// change a row's sum (entry order either way).
inline int block_chunk(int L, int ch) { return L >= 4 ? (ch < 8 ? ch : 8) : ch; }

// Tile of the one-pass block product with L lanes per row: 256 / L rows with
// room for kStreamNnzMax column words when every block of that many rows has
// no more nonzeros (rpb: the operator's row block for kStreamNnzMax), else
// room for kBlockWordsLarge words and as many rows as that allows (rpb_l),
// at most 256 / L.  Both row counts are powers of two, so a tile is an
// aligned part of a block that fits.
struct BlockTile {
    int rows;
    bool large;
};
inline BlockTile block_tile(int L, int rpb, int rpb_l) {
    const int full = 256 / L;
    if (rpb >= full) return {full, false};
    return {rpb_l < full ? (rpb_l > 1 ? rpb_l : 1) : full, true};
}

// Y[r] = d_r X[r] + sum over the row's entries of +-|t| X[col] for one tile
// of rows [rbeg, rend) of an n-row block of NV vectors (row-major, 16-byte
// aligned) in a single pass: rend - rbeg <= 256 / L with L = NV / (16 /
// sizeof T) lanes per row, each lane 16 bytes of the gathered row (float4 /
// double2), and the tile's entries <= WMAX.  Every thread first issues its
// loads -- its row's pointers, diagonal and own X row, the tile's first and
// last pointers, the amplitude table -- then the tile's column words are
// loaded together (coalesced, unconditional loads on clamped addresses) into
// LDS, and after one barrier each row reads its words from LDS, CH at a
// time, and issues their gathers; sum in entry order.  Two dependent global
// round trips before the gathers.  Every thread of the workgroup must call
// it (barrier).
template <typename T, int NV, int CH, int WMAX>
__device__ __forceinline__ void block_csr_v_tile(const int64_t *__restrict__ rowptr,
                                                 const uint32_t *__restrict__ colw,
                                                 const DevModel *__restrict__ m,
                                                 const double *__restrict__ diag,
                                                 const T *__restrict__ x, T *__restrict__ y,
                                                 int64_t rbeg, int64_t rend) {
    // 16 bytes of a row as a clang vector (loads and stores through global
    // pointers; element-wise arithmetic)
    using V = T __attribute__((ext_vector_type(Vec16<T>::n)));
    constexpr int L = NV / Vec16<T>::n;
    static_assert(L >= 1 && L * Vec16<T>::n == NV, "NV must be a multiple of the vector width");
    constexpr int DEPTH = WMAX / 256;
    static_assert(DEPTH * 256 == WMAX, "whole words per thread");
    __shared__ T vtab[kMaxClasses];
    __shared__ uint32_t wl[WMAX];
    const int t = threadIdx.x, lane = t % L;
    // every load and store as a global one (the many-run kernel passes
    // pointers read from its run table)
    const GPtr<const V> xv4 = (GPtr<const V>)x;
    const GPtr<V> yv4 = (GPtr<V>)y;
    const GPtr<const int64_t> rp = (GPtr<const int64_t>)rowptr;
    const GPtr<const uint32_t> cw = (GPtr<const uint32_t>)colw;
    const GPtr<const double> dg = (GPtr<const double>)diag;
    const GPtr<const DevModel> mg = (GPtr<const DevModel>)m;
    const int64_t r = rbeg + t / L;
    const bool own = r < rend;
    const int64_t rr = own ? r : rend - 1;
    const int64_t e0 = rp[rbeg], eT = rp[rend];
    const int64_t b0 = rp[rr], e1 = rp[rr + 1];
    const T d = (T)dg[rr];
    const V xr = xv4[rr * L + lane];
    if (t < kMaxClasses) vtab[t] = (T)mg->vtab[t];
    const uint32_t cmask = mg->col_mask, cbits = mg->col_bits;
    const int cnt = (int)(eT - e0);
    if (cnt > 0) {   // uniform over the workgroup
        uint32_t w[DEPTH];
#pragma unroll
        for (int j = 0; j < DEPTH; j++) w[j] = cw[e0 + min(t + j * 256, cnt - 1)];
#pragma unroll
        for (int j = 0; j < DEPTH; j++)
            if (t + j * 256 < cnt) wl[t + j * 256] = w[j];
    }
    __syncthreads();
    if (!own) return;
    V acc = d * xr;
    const int s1 = (int)(e1 - e0);
    for (int base = (int)(b0 - e0); base < s1; base += CH) {
        uint32_t wj[CH];
        V xg[CH];
#pragma unroll
        for (int j = 0; j < CH; j++) wj[j] = base + j < s1 ? wl[base + j] : 0u;
#pragma unroll
        for (int j = 0; j < CH; j++) {
            xg[j] = V(0);
            if (base + j < s1) xg[j] = xv4[(int64_t)(wj[j] & cmask) * L + lane];
        }
#pragma unroll
        for (int j = 0; j < CH; j++) {
            if (base + j < s1) {
                const T v = vtab[(wj[j] & 0x7fffffffu) >> cbits];
                acc += ((wj[j] >> 31) ? -v : v) * xg[j];
            }
        }
    }
    yv4[r * L + lane] = acc;
}

}  // namespace mcd
