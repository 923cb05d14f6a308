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

// Grid-wide sum by the "last block finishes" pattern: every block deposits
// its partial, the block that arrives last adds all partials in index order
// and writes *out.  Deterministic for a fixed grid.  `counter` must be zero
// on entry and is zero again on exit.  Every thread of every block calls it
// with its block's value in thread 0.
template <int BS>
__device__ __forceinline__ void grid_sum_last(double block_val, int nblocks, double *partials,
                                              unsigned int *counter, double *out) {
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = block_val;
        __threadfence();
        unsigned int prev = atomicAdd(counter, 1u);
        is_last = (prev == (unsigned int)nblocks - 1u);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        double s = 0.0;
        for (int i = threadIdx.x; i < nblocks; i += BS)
            s += __hip_atomic_load(&partials[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = block_sum<BS>(s);
        if (threadIdx.x == 0) {
            *out = s;
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace mcd
