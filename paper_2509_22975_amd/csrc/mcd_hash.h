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

// Lanczos start value of a basis state: 2u - 1 with u the top 53 bits of
// splitmix64's first output from the state (seed XOR key).
__device__ __forceinline__ double start_value(uint64_t key, uint64_t seed) {
    uint64_t z = (key ^ seed) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

}  // namespace mcd
