// Open-addressing hash of the basis (key -> row), shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mcd_internal.h"

namespace mcd {

__device__ __forceinline__ uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Row of `key`, or -1 if the state is not in the basis (linear probing).
__device__ __forceinline__ int64_t hash_find(const HashSlot *__restrict__ h, uint64_t mask,
                                             uint64_t key) {
    uint64_t p = mix64(key) & mask;
    for (;;) {
        const uint64_t k = h[p].key;
        if (k == key) return h[p].val;
        if (k == kEmpty) return -1;
        p = (p + 1) & mask;
    }
}

}  // namespace mcd
