// Deterministic wavefront / workgroup / grid reductions for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace mcd {

// Scale factor held on the device: mode 0 -> *p, mode 1 -> 1/sqrt(*p)
// (p = a squared norm), p == nullptr -> 1.
__device__ __forceinline__ double scale_from(const double *p, int mode) {
    if (p == nullptr) return 1.0;
    const double v = *p;
    if (mode == 0) return v;
    return v > 0.0 ? 1.0 / sqrt(v) : 0.0;
}

// Sum over a 64-lane wavefront (fixed butterfly order, result in lane 0).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the workgroup; the result is valid in thread 0.  Every thread of
// the block must call it (it synchronises).
template <int BS>
__device__ __forceinline__ double block_sum(double v) {
    static_assert(BS % 64 == 0, "block size must be a multiple of the wavefront");
    __shared__ double red[BS / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < BS / 64; i++) r += red[i];
    }
    __syncthreads();
    return r;
}

// Grid-wide sums are two-phase: every workgroup stores its partial (thread 0)
// and a one-workgroup kernel adds the partials in index order.  The kernel
// boundary orders the stores; no fences or atomics, deterministic for a fixed
// grid.  (A "last workgroup finishes" scheme needs an agent-scope release
// fence per workgroup, which on CDNA writes back the L2 and costs far more
// than the extra launch.)
template <int BS>
__device__ __forceinline__ void store_partial(double block_val, double *partials) {
    if (threadIdx.x == 0) partials[blockIdx.x] = block_val;
}

// out[0] = sum_i partials[i]: one workgroup; thread t adds t, t + BS, ...
// into four accumulators (k mod 4, a last partial group into the first) in
// index order, then the workgroup sum.  Up to 32 partials per thread are all
// loaded before the first add (one memory round trip instead of one per
// group of four); the order of the additions is the same either way.
template <int BS>
__global__ __launch_bounds__(BS) void k_finalize_sum(int n, const double *__restrict__ partials,
                                                     double *__restrict__ out) {
    constexpr int KMAX = 32;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int t = threadIdx.x;
    if (n > 0 && n <= KMAX * BS) {
        double v[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; k++) v[k] = partials[min(t + k * BS, n - 1)];
        const int K = t < n ? (n - 1 - t) / BS + 1 : 0;
        const int K4 = K & ~3;
#pragma unroll
        for (int g = 0; g < KMAX / 4; g++) {
            if (4 * g < K4) {
                s0 += v[4 * g];
                s1 += v[4 * g + 1];
                s2 += v[4 * g + 2];
                s3 += v[4 * g + 3];
            }
        }
#pragma unroll
        for (int k = 0; k < KMAX; k++)
            if (k >= K4 && k < K) s0 += v[k];
    } else {
        int i = t;
        for (; i + 3 * BS < n; i += 4 * BS) {
            s0 += partials[i];
            s1 += partials[i + BS];
            s2 += partials[i + 2 * BS];
            s3 += partials[i + 3 * BS];
        }
        for (; i < n; i += BS) s0 += partials[i];
    }
    const double s = block_sum<BS>((s0 + s1) + (s2 + s3));
    if (threadIdx.x == 0) *out = s;
}

}  // namespace mcd
