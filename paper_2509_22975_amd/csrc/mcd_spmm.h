// Block product of the packed CSR with 16-byte gathers, as a device
// function over a range of rows, shared by the one-operator kernel
// (mcd_op.hip) and the kernel that serves many band runs in one launch
// (mcd_band.hip).
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
__device__ __forceinline__ float4 vscale(float a, const float4 &x) {
    return make_float4(a * x.x, a * x.y, a * x.z, a * x.w);
}
__device__ __forceinline__ double2 vscale(double a, const double2 &x) {
    return make_double2(a * x.x, a * x.y);
}
__device__ __forceinline__ void vscale_add(float4 &acc, float a, const float4 &x) {
    acc.x += a * x.x;
    acc.y += a * x.y;
    acc.z += a * x.z;
    acc.w += a * x.w;
}
__device__ __forceinline__ void vscale_add(double2 &acc, double a, const double2 &x) {
    acc.x += a * x.x;
    acc.y += a * x.y;
}

// Launch shape of the row-parallel block product with L lanes per row
// (measured on gfx950, C2 basis, 8 and 16 vectors): row tiles that keep all
// 256 threads busy at L <= 2 and 64-row tiles above; at most 8 gathers in
// flight per lane at L >= 4 (ch: words per chunk from the mean row length).
// Neither changes a row's sum (entry order either way).
inline int block_rows_per_tile(int L) { return L <= 2 ? 256 / L : 64; }
inline int block_chunk(int L, int ch) { return L >= 4 ? (ch < 8 ? ch : 8) : ch; }

// Y[r] = d_r X[r] + sum over the row's entries of +-|t| X[col] for the rows
// [rbeg, rend) of an n-row block of NV vectors (row-major, 16-byte aligned):
// L = NV / (16 / sizeof T) lanes per row, each lane 16 bytes of the gathered
// row (float4 / double2); the row's words loaded CH at a time (one coalesced
// access) and broadcast by lane shuffles, CH gathers in flight; sum in entry
// order.  Every thread of the workgroup must call it (the amplitude table
// goes through LDS behind a barrier).
template <typename T, int NV, int CH>
__device__ __forceinline__ void block_csr_v_rows(const int64_t *__restrict__ rowptr,
                                                 const uint32_t *__restrict__ colw,
                                                 const DevModel *__restrict__ m,
                                                 const double *__restrict__ diag,
                                                 const T *__restrict__ x, T *__restrict__ y,
                                                 int64_t rbeg, int64_t rend) {
    using V = typename Vec16<T>::type;
    constexpr int L = NV / Vec16<T>::n;
    static_assert(L >= 1 && L * Vec16<T>::n == NV, "NV must be a multiple of the vector width");
    __shared__ T vtab[kMaxClasses];
    if (threadIdx.x < kMaxClasses) vtab[threadIdx.x] = (T)m->vtab[threadIdx.x];
    __syncthreads();
    const uint32_t cmask = m->col_mask, cbits = m->col_bits;
    constexpr int RPB = 256 / L;
    constexpr int WPL = (CH + L - 1) / L;
    const int lane = threadIdx.x % L;
    const V *__restrict__ xv4 = reinterpret_cast<const V *>(x);
    V *__restrict__ yv4 = reinterpret_cast<V *>(y);
    for (int64_t r = rbeg + threadIdx.x / L; r < rend; r += RPB) {
        const T d = (T)diag[r];
        V acc = vscale(d, xv4[r * L + lane]);
        const int64_t e1 = rowptr[r + 1];
        // the words of the row's first two chunks are loaded at once (a row
        // of up to 2 CH entries waits for one word load, not two)
        uint32_t mw2[2 * WPL];
        {
            const int64_t b0 = rowptr[r];
#pragma unroll
            for (int c = 0; c < 2; c++)
#pragma unroll
                for (int q = 0; q < WPL; q++) {
                    const int64_t e = b0 + c * CH + q * L + lane;
                    mw2[c * WPL + q] = (q * L + lane < CH && e < e1) ? colw[e] : 0u;
                }
        }
        int chunk = 0;
        for (int64_t base = rowptr[r]; base < e1; base += CH, chunk++) {
            uint32_t mw[WPL];
            if (chunk < 2) {
#pragma unroll
                for (int q = 0; q < WPL; q++) mw[q] = chunk == 0 ? mw2[q] : mw2[WPL + q];
            } else {
#pragma unroll
                for (int q = 0; q < WPL; q++) {
                    const int64_t e = base + q * L + lane;
                    mw[q] = (q * L + lane < CH && e < e1) ? colw[e] : 0u;
                }
            }
            uint32_t wj[CH];
            V xg[CH];
#pragma unroll
            for (int j = 0; j < CH; j++) {
                wj[j] = (uint32_t)__shfl((int)mw[j / L], j % L, L);
                xg[j] = (base + j < e1) ? xv4[(int64_t)(wj[j] & cmask) * L + lane] : V{};
            }
#pragma unroll
            for (int j = 0; j < CH; j++) {
                if (base + j < e1) {
                    const T v = vtab[(wj[j] & 0x7fffffffu) >> cbits];
                    vscale_add(acc, (wj[j] >> 31) ? -v : v, xg[j]);
                }
            }
        }
        yv4[r * L + lane] = acc;
    }
}

}  // namespace mcd
