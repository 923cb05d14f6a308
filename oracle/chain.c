/* Oracle Metropolis chain that draws the truncated basis F~ (plain C).
 *
 * TEST INFRASTRUCTURE ONLY: built by the oracle and called from the tests,
 * never linked into the product library.
 *
 * The sampling follows the paper's variant 1 acceptance (Sec. Other sampling
 * methods, Eq. boltzmann_factor2: a ratio of Boltzmann factors) combined with
 * variant 2's proposal (one random hop per step), weighted by the diagonal
 * energy with inverse temperature beta_s.  Every draw comes from Vigna's
 * splitmix64 generator seeded with `seed` (two draws per step):
 *
 *   r0, r1 = next(), next()
 *   m = (hi32(r0) * M) >> 32, M = 4 * n_bonds: bond = m >> 2,
 *       spin = (m >> 1) & 1 (0 = up), dir = m & 1 (0: i -> j, 1: j -> i)
 *   the hop is invalid (a rejected step) unless the source orbital is
 *       occupied and the target empty in that spin string
 *   dE = (eps[dst] - eps[src]) + (U[dst]*o[dst] - U[src]*o[src]),
 *       o = other-spin occupation, evaluated in that order in float64
 *   accept iff dE <= 0 or u < exp(-beta_s * dE), u = (r1 >> 11) * 2^-53
 *
 * Recording: after the first burn_in steps the current state is inserted
 * into the set after every step; the chain stops when the set holds n_f
 * states or after max_steps steps in total.  The set is returned sorted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_state;

static uint64_t sm_next(void) {
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t *slot;
    uint64_t mask;
    int64_t count;
} set_t;

static uint64_t hash64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    return k;
}

static void set_insert(set_t *s, uint64_t key) {
    uint64_t h = hash64(key) & s->mask;
    for (;;) {
        if (s->slot[h] == key) return;
        if (s->slot[h] == ~0ULL) {
            s->slot[h] = key;
            s->count++;
            return;
        }
        h = (h + 1) & s->mask;
    }
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y);
}

int64_t oracle_chain(int n_bonds, const int *bi, const int *bj, const double *U,
                     const double *eps, uint64_t start, uint64_t seed, double beta_s,
                     int64_t burn_in, int64_t max_steps, int64_t n_f, uint64_t *out,
                     int64_t *steps_done) {
    uint64_t cap = 1;
    while (cap < (uint64_t)(2 * n_f + 2)) cap <<= 1;
    set_t s;
    s.slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!s.slot) return -1;
    memset(s.slot, 0xff, cap * sizeof(uint64_t));
    s.mask = cap - 1;
    s.count = 0;

    sm_state = seed;
    uint64_t up = start >> 32, dn = start & 0xffffffffULL;
    const uint64_t M = 4ULL * (uint64_t)n_bonds;
    int64_t step = 0;
    while (step < max_steps && s.count < n_f) {
        uint64_t r0 = sm_next(), r1 = sm_next();
        uint64_t m = ((r0 >> 32) * M) >> 32;
        int b = (int)(m >> 2), spin = (int)((m >> 1) & 1), dir = (int)(m & 1);
        int i = bi[b] < bj[b] ? bi[b] : bj[b];
        int j = bi[b] < bj[b] ? bj[b] : bi[b];
        int src = dir == 0 ? i : j, dst = dir == 0 ? j : i;
        uint64_t *sv = spin == 0 ? &up : &dn;
        uint64_t other = spin == 0 ? dn : up;
        if (((*sv >> src) & 1ULL) && !((*sv >> dst) & 1ULL)) {
            double o_dst = (double)((other >> dst) & 1ULL);
            double o_src = (double)((other >> src) & 1ULL);
            double dE = (eps[dst] - eps[src]) + (U[dst] * o_dst - U[src] * o_src);
            double u = (double)(r1 >> 11) * (1.0 / 9007199254740992.0);
            if (dE <= 0.0 || u < exp(-beta_s * dE)) {
                *sv ^= (1ULL << src) | (1ULL << dst);
            }
        }
        step++;
        if (step > burn_in) set_insert(&s, (up << 32) | dn);
    }
    int64_t k = 0;
    for (uint64_t h = 0; h < cap; h++)
        if (s.slot[h] != ~0ULL) out[k++] = s.slot[h];
    qsort(out, (size_t)k, sizeof(uint64_t), cmp_u64);
    free(s.slot);
    *steps_done = step;
    return k;
}

/* Visit counts of a long chain over an enumerated sector (stationarity pin):
 * counts[r] = number of recorded steps spent in keys[r]. */
int oracle_chain_histogram(int n_bonds, const int *bi, const int *bj, const double *U,
                           const double *eps, uint64_t start, uint64_t seed, double beta_s,
                           int64_t burn_in, int64_t steps, const uint64_t *keys, int64_t n_keys,
                           int64_t *counts) {
    sm_state = seed;
    uint64_t up = start >> 32, dn = start & 0xffffffffULL;
    const uint64_t M = 4ULL * (uint64_t)n_bonds;
    for (int64_t step = 1; step <= burn_in + steps; step++) {
        uint64_t r0 = sm_next(), r1 = sm_next();
        uint64_t m = ((r0 >> 32) * M) >> 32;
        int b = (int)(m >> 2), spin = (int)((m >> 1) & 1), dir = (int)(m & 1);
        int i = bi[b] < bj[b] ? bi[b] : bj[b];
        int j = bi[b] < bj[b] ? bj[b] : bi[b];
        int src = dir == 0 ? i : j, dst = dir == 0 ? j : i;
        uint64_t *sv = spin == 0 ? &up : &dn;
        uint64_t other = spin == 0 ? dn : up;
        if (((*sv >> src) & 1ULL) && !((*sv >> dst) & 1ULL)) {
            double o_dst = (double)((other >> dst) & 1ULL);
            double o_src = (double)((other >> src) & 1ULL);
            double dE = (eps[dst] - eps[src]) + (U[dst] * o_dst - U[src] * o_src);
            double u = (double)(r1 >> 11) * (1.0 / 9007199254740992.0);
            if (dE <= 0.0 || u < exp(-beta_s * dE)) *sv ^= (1ULL << src) | (1ULL << dst);
        }
        if (step > burn_in) {
            uint64_t key = (up << 32) | dn;
            int64_t lo = 0, hi = n_keys - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (keys[mid] < key) lo = mid + 1; else hi = mid;
            }
            if (keys[lo] != key) return -1;
            counts[lo]++;
        }
    }
    return 0;
}
