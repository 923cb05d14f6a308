// The truncated basis F~ (Sec. Subspace of the ground state; Sec. Other
// sampling methods).
//
// Full sector: every key of (n_up, n_dn), produced in sorted order on the GPU
// by unranking combinations (combinatorial number system, up string major).
//
// Chain: a Metropolis chain over the sector, one random hop per step,
// accepted with the Boltzmann ratio of the diagonal energy.  A Markov chain
// is sequential, so the host walks it; it only emits the steps at which the
// state changes (plus the first recorded step).  The GPU does the rest: a
// hash table keeps, for every distinct state, the earliest step it was
// recorded at (atomicMin); the first n_f distinct states in order of first
// visit are exactly the states a sequential "stop at n_f" run would hold;
// they are selected by sorting first-visit steps and then sorted by key.
#include <hipcub/hipcub.hpp>
#include <math.h>

#include <algorithm>
#include <vector>

#include "mcd_internal.h"

namespace mcd {

struct Binom {
    uint64_t c[MCD_MAX_ORB + 1][MCD_MAX_ORB + 1];
};

static void fill_binom(Binom &b) {
    memset(&b, 0, sizeof(b));
    for (int n = 0; n <= MCD_MAX_ORB; n++) {
        b.c[n][0] = 1;
        for (int k = 1; k <= n; k++) b.c[n][k] = b.c[n - 1][k - 1] + (k <= n - 1 ? b.c[n - 1][k] : 0);
    }
}

// The r-th smallest n-bit string with k ones (r counted from 0).
__device__ __forceinline__ uint32_t unrank(uint64_t r, int n, int k, const Binom *__restrict__ B) {
    uint32_t s = 0;
    for (int i = n - 1; i >= 0 && k > 0; i--) {
        const uint64_t below = B->c[i][k];   // strings using only bits < i
        if (r >= below) {
            s |= 1u << i;
            r -= below;
            k--;
        }
    }
    return s;
}

__global__ void k_enumerate(uint64_t total, uint64_t n_dn_states, int n, int nu, int nd,
                            const Binom *__restrict__ B, uint64_t *__restrict__ keys) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const uint64_t ru = q / n_dn_states, rd = q % n_dn_states;
    keys[q] = ((uint64_t)unrank(ru, n, nu, B) << 32) | unrank(rd, n, nd, B);
}

struct VisitSlot {
    unsigned long long key;
    unsigned long long step;
};

__device__ __forceinline__ uint64_t vmix(uint64_t k) {
    k ^= k >> 31;
    k *= 0x7fb5d329728ea185ull;
    k ^= k >> 27;
    k *= 0x81dadef4bc2dd44dull;
    k ^= k >> 33;
    return k;
}

__global__ void k_visit_insert(int64_t m, const uint64_t *__restrict__ ev_key,
                               const uint64_t *__restrict__ ev_step, VisitSlot *tab, uint64_t mask,
                               unsigned long long *distinct) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t key = ev_key[i];
    uint64_t p = vmix(key) & mask;
    for (;;) {
        const unsigned long long prev = atomicCAS(&tab[p].key, (unsigned long long)kEmpty,
                                                  (unsigned long long)key);
        if (prev == kEmpty) atomicAdd(distinct, 1ull);
        if (prev == kEmpty || prev == key) {
            atomicMin(&tab[p].step, (unsigned long long)ev_step[i]);
            return;
        }
        p = (p + 1) & mask;
    }
}

__global__ void k_visit_compact(uint64_t cap, const VisitSlot *__restrict__ tab,
                                uint64_t *__restrict__ steps, uint64_t *__restrict__ keys,
                                unsigned long long *cnt) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= cap) return;
    const VisitSlot v = tab[p];
    if (v.key == kEmpty) return;
    const unsigned long long at = atomicAdd(cnt, 1ull);
    steps[at] = v.step;
    keys[at] = v.key;
}

// splitmix64 (Vigna): the chain's random stream.
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// Host walker of the chain: advances `nsteps` steps and appends (step, key)
// whenever a recorded step holds a state different from the previous record.
struct ChainWalker {
    const mcd_model *m;
    std::vector<int> lo, hi;
    uint64_t up, dn;
    SplitMix rng;
    double beta;
    int64_t step = 0, burn_in;
    bool have_record = false;

    void run(int64_t nsteps, std::vector<uint64_t> &ek, std::vector<uint64_t> &es) {
        const uint64_t M = 4ull * (uint64_t)lo.size();
        for (int64_t it = 0; it < nsteps; it++) {
            const uint64_t r0 = rng.next(), r1 = rng.next();
            const uint64_t pick = ((r0 >> 32) * M) >> 32;
            const int b = (int)(pick >> 2);
            const bool spin_dn = ((pick >> 1) & 1ull) != 0;
            const bool rev = (pick & 1ull) != 0;
            const int src = rev ? hi[b] : lo[b], dst = rev ? lo[b] : hi[b];
            uint64_t &mine = spin_dn ? dn : up;
            const uint64_t other = spin_dn ? up : dn;
            bool moved = false;
            if (((mine >> src) & 1ull) != 0 && ((mine >> dst) & 1ull) == 0) {
                const double od = (double)((other >> dst) & 1ull);
                const double os = (double)((other >> src) & 1ull);
                const double dE = (m->eps[dst] - m->eps[src]) + (m->U[dst] * od - m->U[src] * os);
                const double u = (double)(r1 >> 11) * (1.0 / 9007199254740992.0);
                if (dE <= 0.0 || u < exp(-beta * dE)) {
                    mine ^= (1ull << src) | (1ull << dst);
                    moved = true;
                }
            }
            step++;
            if (step > burn_in && (moved || !have_record)) {
                ek.push_back((up << 32) | dn);
                es.push_back((uint64_t)step);
                have_record = true;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// The paper's step sampler (Sec. Subspace of the ground state, numbered step
// procedure; acceptance Eq. boltzmann_factor).  One step on the GPU:
//   k_bfs_expand     every (frontier parent, hop) pair: possible? accepted
//                    with probability table[n_U] (n_U on the interacting
//                    orbitals) against a counter-based uniform; accepted
//                    images compacted with one atomic per wavefront, tagged
//                    with their order (parent rank * H + hop);
//   radix sort by key, k_bfs_heads / scan / k_bfs_unique: each state once,
//                    with its first order, and whether it is already in F~;
//   the unique states (sorted by key) are the next frontier; the new ones,
//   radix-sorted by order, join F~ until it holds n_f states.
struct BfsHop {
    uint32_t src, dst, spin, pad;
};

__device__ __forceinline__ uint64_t bfs_mix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_bfs_expand(int64_t total, int H, const uint64_t *__restrict__ F,
                             const BfsHop *__restrict__ hops, uint32_t umask,
                             const double *__restrict__ table, uint64_t seed, uint64_t step,
                             uint64_t *__restrict__ out_key, uint64_t *__restrict__ out_ord,
                             unsigned long long *counter) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool acc = false;
    uint64_t y = 0;
    if (idx < total) {
        const int64_t p = idx / H;
        const int h = (int)(idx % H);
        const uint64_t x = F[p];
        const uint32_t up = (uint32_t)(x >> 32), dn = (uint32_t)x;
        const BfsHop hp = hops[h];
        const uint32_t sv = hp.spin ? dn : up;
        if (((sv >> hp.src) & 1u) && !((sv >> hp.dst) & 1u)) {
            const uint32_t s2 = sv ^ ((1u << hp.src) | (1u << hp.dst));
            y = hp.spin ? (((uint64_t)up << 32) | s2) : (((uint64_t)s2 << 32) | dn);
            const int nu = __popc((uint32_t)(y >> 32) & (uint32_t)y & umask);
            const uint64_t z = bfs_mix(bfs_mix(bfs_mix(seed ^ (step * 0x9E3779B97F4A7C15ull)) ^ x) ^
                                       (uint64_t)h);
            const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            acc = u < table[nu];
        }
    }
    // one atomic per wavefront
    const unsigned long long ball = __ballot(acc);
    const int lane = __lane_id();
    unsigned long long base = 0;
    if (lane == __ffsll((long long)ball) - 1 && ball != 0ull) base = atomicAdd(counter, (unsigned long long)__popcll(ball));
    base = __shfl(base, __ffsll((long long)ball) - 1 >= 0 ? __ffsll((long long)ball) - 1 : 0, 64);
    if (acc) {
        const unsigned long long pos = base + __popcll(ball & ((1ull << lane) - 1ull));
        out_key[pos] = y;
        out_ord[pos] = (uint64_t)idx;
    }
}

__global__ void k_bfs_heads(int64_t m, const uint64_t *__restrict__ k, int64_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) flag[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
    if (i == m) flag[m] = 0;
}

__device__ __forceinline__ bool set_has(const uint64_t *__restrict__ t, uint64_t mask, uint64_t key) {
    uint64_t p = vmix(key) & mask;
    for (;;) {
        const uint64_t v = t[p];
        if (v == key) return true;
        if (v == kEmpty) return false;
        p = (p + 1) & mask;
    }
}

__global__ void k_bfs_unique(int64_t m, const uint64_t *__restrict__ k, const uint64_t *__restrict__ ord,
                             const int64_t *__restrict__ pos, const uint64_t *__restrict__ set,
                             uint64_t smask, uint64_t *__restrict__ ukey, uint64_t *__restrict__ uord,
                             int64_t *__restrict__ isnew) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (!(i == 0 || k[i] != k[i - 1])) return;
    uint64_t best = ord[i];
    for (int64_t j = i + 1; j < m && k[j] == k[i]; j++) best = min(best, ord[j]);
    const int64_t q = pos[i];
    ukey[q] = k[i];
    uord[q] = best;
    isnew[q] = set_has(set, smask, k[i]) ? 0 : 1;
}

__global__ void k_bfs_compact_new(int64_t u, const uint64_t *__restrict__ ukey,
                                  const uint64_t *__restrict__ uord, const int64_t *__restrict__ isnew,
                                  const int64_t *__restrict__ npos, uint64_t *__restrict__ nkey,
                                  uint64_t *__restrict__ nord) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= u || !isnew[i]) return;
    nkey[npos[i]] = ukey[i];
    nord[npos[i]] = uord[i];
}

__global__ void k_set_insert(int64_t m, const uint64_t *__restrict__ keys, uint64_t *set,
                             uint64_t mask, uint64_t *__restrict__ list, int64_t list0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t key = keys[i];
    uint64_t p = vmix(key) & mask;
    for (;;) {
        const unsigned long long prev = atomicCAS((unsigned long long *)&set[p],
                                                  (unsigned long long)kEmpty, (unsigned long long)key);
        if (prev == kEmpty || prev == key) break;
        p = (p + 1) & mask;
    }
    list[list0 + i] = key;
}


// Map the bits of `rel` (positions counted among the set bits of `freem`,
// lowest first) to absolute positions.
__device__ __forceinline__ uint32_t spread_bits(uint32_t rel, uint32_t freem) {
    uint32_t out = 0;
    int j = 0;
    while (freem) {
        const uint32_t low = freem & (~freem + 1u);
        if ((rel >> j) & 1u) out |= low;
        freem ^= low;
        j++;
    }
    return out;
}

// Level n_U = k of the (nu, nd) sector on n orbitals: state q = (i1, i2, i3)
// in mixed radix -> k doubly occupied sites (rank i1 among C(n, k)), nu - k
// up-only sites among the other n - k (rank i2), nd - k down-only sites among
// the n - nu sites still empty (rank i3).
__global__ void k_enum_level(uint64_t count, int n, int nu, int nd, int k,
                             const Binom *__restrict__ B, uint64_t *__restrict__ out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const uint64_t c3 = B->c[n - nu][nd - k], c2 = B->c[n - k][nu - k];
    const uint64_t i3 = q % c3, t = q / c3;
    const uint64_t i2 = t % c2, i1 = t / c2;
    const uint32_t all = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
    const uint32_t D = unrank(i1, n, k, B);
    const uint32_t A = spread_bits(unrank(i2, n - k, nu - k, B), all & ~D);
    const uint32_t Bd = spread_bits(unrank(i3, n - nu, nd - k, B), all & ~(D | A));
    out[q] = ((uint64_t)(D | A) << 32) | (uint64_t)(D | Bd);
}

static int build_bfs(const mcd_model *model, const mcd_basis_cfg *cfg, uint64_t *keys_dev,
                     int64_t cap, int64_t *n_out, int64_t *steps_out, mcd_ws *ws, hipStream_t s) {
    const Alloc al{ws};
    const uint64_t lim = model->n_orb >= 32 ? 0xffffffffull : ((1ull << model->n_orb) - 1ull);
    const uint64_t su = cfg->start_key >> 32, sd = cfg->start_key & 0xffffffffull;
    MCD_REQUIRE((su & ~lim) == 0 && (sd & ~lim) == 0 && __builtin_popcountll(su) == cfg->n_up &&
                    __builtin_popcountll(sd) == cfg->n_dn,
                MCD_E_SECTOR, "start key is not in the (%d, %d) sector", cfg->n_up, cfg->n_dn);
    MCD_REQUIRE(model->n_bonds >= 1 && cfg->n_f >= 1, MCD_E_INVALID, "need bonds and n_f >= 1");
    MCD_REQUIRE(cfg->n_f <= cap, MCD_E_CAPACITY, "cap %lld < n_f %lld", (long long)cap,
                (long long)cfg->n_f);
    // common U of the interacting orbitals, acceptance table exp(-beta U k)
    double U0 = 0.0;
    uint32_t umask = 0;
    for (int i = 0; i < model->n_orb; i++) {
        if (model->U[i] == 0.0) continue;
        MCD_REQUIRE(U0 == 0.0 || model->U[i] == U0, MCD_E_INVALID,
                    "the step sampler needs one common U on the interacting orbitals");
        U0 = model->U[i];
        umask |= 1u << i;
    }
    double table[MCD_MAX_ORB + 1];
    for (int k = 0; k <= MCD_MAX_ORB; k++) table[k] = exp(-cfg->beta_s * U0 * (double)k);
    const int H = 4 * model->n_bonds;
    std::vector<BfsHop> hh(H);
    for (int h = 0; h < H; h++) {
        const int b = h >> 2;
        const uint32_t i = (uint32_t)std::min(model->bond_i[b], model->bond_j[b]);
        const uint32_t j = (uint32_t)std::max(model->bond_i[b], model->bond_j[b]);
        const bool rev = (h & 1) != 0;
        hh[h] = BfsHop{rev ? j : i, rev ? i : j, (uint32_t)((h >> 1) & 1), 0u};
    }
    const int64_t nf = cfg->n_f;
    uint64_t smask = 1023;
    while (smask + 1 < (uint64_t)(4 * nf)) smask = (smask << 1) | 1;
    // buffers (grown on demand)
    BfsHop *d_hops = nullptr;
    double *d_table = nullptr;
    uint64_t *set = nullptr, *F = nullptr, *ak = nullptr, *ao = nullptr, *bk = nullptr, *bo = nullptr;
    uint64_t *uk = nullptr, *uo = nullptr, *nk = nullptr, *no = nullptr, *nk2 = nullptr, *no2 = nullptr;
    int64_t *flag = nullptr, *pos = nullptr, *isnew = nullptr, *npos = nullptr;
    unsigned long long *cnt = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int64_t capA = 0, capF = 0, capM = 0;
    auto cleanup = [&]() {
        for (void *p : {(void *)d_hops, (void *)d_table, (void *)set, (void *)F, (void *)ak,
                        (void *)ao, (void *)bk, (void *)bo, (void *)uk, (void *)uo, (void *)nk,
                        (void *)no, (void *)nk2, (void *)no2, (void *)flag, (void *)pos,
                        (void *)isnew, (void *)npos, (void *)cnt, tmp})
            if (p) (void)dfree(p, al);
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
    auto grow = [&](void **p, int64_t bytes) -> hipError_t {
        if (*p) {
            hipError_t e = dfree(*p, al);
            if (e != hipSuccess) return e;
        }
        *p = nullptr;
        return dmalloc(p, std::max<int64_t>(bytes, 8), al);
    };
    auto need_tmp = [&](size_t b) -> hipError_t {
        if (b <= tmp_bytes) return hipSuccess;
        if (tmp) (void)dfree(tmp, al);
        tmp = nullptr;
        tmp_bytes = b;
        return dmalloc((void **)&tmp, b, al);
    };
    CK(dmalloc((void **)&d_hops, H * sizeof(BfsHop), al));
    CK(hipMemcpyAsync(d_hops, hh.data(), H * sizeof(BfsHop), hipMemcpyHostToDevice, s));
    CK(dmalloc((void **)&d_table, sizeof(table), al));
    CK(hipMemcpyAsync(d_table, table, sizeof(table), hipMemcpyHostToDevice, s));
    CK(dmalloc((void **)&set, (smask + 1) * sizeof(uint64_t), al));
    CK(hipMemsetAsync(set, 0xff, (smask + 1) * sizeof(uint64_t), s));
    CK(dmalloc((void **)&cnt, 2 * sizeof(unsigned long long), al));
    // Pre-accepted levels n_U < pre_level, level by level, each sorted by key.
    int64_t npre = 0;
    bool pre_done = false;
    if (cfg->pre_level > 0) {
        const uint32_t all = model->n_orb >= 32 ? 0xffffffffu : ((1u << model->n_orb) - 1u);
        if (umask != all) {
            cleanup();
            set_error("pre-acceptance needs U != 0 on every orbital");
            return MCD_E_INVALID;
        }
        Binom hb;
        fill_binom(hb);
        Binom *db = nullptr;
        uint64_t *lv = nullptr, *lv2 = nullptr;
        auto freelv = [&]() {
            for (void *p : {(void *)db, (void *)lv, (void *)lv2})
                if (p) (void)dfree(p, al);
        };
        const int n = model->n_orb, nu = cfg->n_up, nd = cfg->n_dn;
        if (dmalloc((void **)&db, sizeof(Binom), al) != hipSuccess) {
            cleanup();
            set_error("pre-acceptance: workspace too small for the binomial table");
            return MCD_E_WORKSPACE;
        }
        if (hipMemcpyAsync(db, &hb, sizeof(Binom), hipMemcpyHostToDevice, s) != hipSuccess) {
            freelv();
            cleanup();
            set_error("pre-acceptance: binomial table upload failed");
            return MCD_E_HIP;
        }
        for (int k = 0; k < cfg->pre_level && k <= std::min(nu, nd) && !pre_done; k++) {
            if (nd - k > n - nu) continue;   // no room for the down-only sites
            const uint64_t cnt_k = hb.c[n][k] * hb.c[n - k][nu - k] * hb.c[n - nu][nd - k];
            if (cnt_k == 0) continue;
            if (cnt_k >= (1ull << 31)) {
                freelv();
                cleanup();
                set_error("pre-accepted level n_U = %d has %llu states (limit 2^31)", k,
                          (unsigned long long)cnt_k);
                return MCD_E_CAPACITY;
            }
            const int64_t c = (int64_t)cnt_k;
            int rc = MCD_OK;
            if (dmalloc((void **)&lv, c * 8, al) != hipSuccess ||
                dmalloc((void **)&lv2, c * 8, al) != hipSuccess)
                rc = MCD_E_WORKSPACE;
            if (rc == MCD_OK) {
                hipLaunchKernelGGL(k_enum_level, dim3((unsigned)((c + 255) / 256)), dim3(256), 0,
                                   s, cnt_k, n, nu, nd, k, db, lv);
                size_t b = 0;
                if (hipGetLastError() != hipSuccess ||
                    hipcub::DeviceRadixSort::SortKeys(nullptr, b, lv, lv2, (int)c, 0, 64, s) !=
                        hipSuccess ||
                    need_tmp(b) != hipSuccess)
                    rc = MCD_E_HIP;
                b = tmp_bytes;
                if (rc == MCD_OK &&
                    hipcub::DeviceRadixSort::SortKeys(tmp, b, lv, lv2, (int)c, 0, 64, s) != hipSuccess)
                    rc = MCD_E_HIP;
            }
            const int64_t take = std::min<int64_t>(c, nf - npre);
            if (rc == MCD_OK && hipMemcpyAsync(keys_dev + npre, lv2, take * 8,
                                               hipMemcpyDeviceToDevice, s) != hipSuccess)
                rc = MCD_E_HIP;
            if (rc == MCD_OK && hipStreamSynchronize(s) != hipSuccess) rc = MCD_E_HIP;
            (void)dfree(lv, al);
            (void)dfree(lv2, al);
            lv = lv2 = nullptr;
            if (rc != MCD_OK) {
                freelv();
                cleanup();
                set_error("pre-acceptance: enumerating level n_U = %d failed", k);
                return rc;
            }
            npre += take;
            if (npre >= nf) pre_done = true;
        }
        freelv();
    }
    int64_t nF = 1, nS = 1, step = 0;
    if (npre > 0) {
        // F~ = the pre-accepted states; the frontier = the same set by key
        hipLaunchKernelGGL(k_set_insert, dim3((unsigned)((npre + 255) / 256)), dim3(256), 0, s,
                           npre, keys_dev, set, smask, keys_dev, (int64_t)0);
        CK(hipGetLastError());
        capF = std::max<int64_t>(npre, 1024);
        CK(grow((void **)&F, capF * 8));
        size_t b = 0;
        CK(hipcub::DeviceRadixSort::SortKeys(nullptr, b, keys_dev, F, (int)npre, 0, 64, s));
        CK(need_tmp(b));
        b = tmp_bytes;
        CK(hipcub::DeviceRadixSort::SortKeys(tmp, b, keys_dev, F, (int)npre, 0, 64, s));
        nF = nS = npre;
        if (pre_done) nF = 0;
    } else {
        // F~ starts with the start state; the frontier too
        CK(hipMemcpyAsync(keys_dev, &cfg->start_key, sizeof(uint64_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_set_insert, dim3(1), dim3(64), 0, s, (int64_t)1, keys_dev, set,
                           smask, keys_dev, (int64_t)0);
        capF = 1024;
        CK(grow((void **)&F, capF * 8));
        CK(hipMemcpyAsync(F, &cfg->start_key, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    }
    while (nS < nf && step < cfg->max_steps) {
        step++;
        if (nF == 0) {   // refill the frontier with all of F~ (sorted)
            if (capF < nS) {
                capF = nS;
                CK(grow((void **)&F, capF * 8));
            }
            size_t b = 0;
            CK(hipcub::DeviceRadixSort::SortKeys(nullptr, b, keys_dev, F, (int)nS, 0, 64, s));
            CK(need_tmp(b));
            b = tmp_bytes;
            CK(hipcub::DeviceRadixSort::SortKeys(tmp, b, keys_dev, F, (int)nS, 0, 64, s));
            nF = nS;
        }
        const int64_t total = nF * (int64_t)H;
        if (capA < total) {       // expansion output: one slot per (parent, hop)
            capA = total;
            for (uint64_t **p : {&ak, &ao}) CK(grow((void **)p, capA * 8));
        }
        CK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_bfs_expand, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                           total, H, F, d_hops, umask, d_table, cfg->seed, (uint64_t)step, ak, ao,
                           cnt);
        CK(hipGetLastError());
        unsigned long long na = 0;
        CK(hipMemcpyAsync(&na, cnt, sizeof(na), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        const int64_t m = (int64_t)na;
        if (m == 0) {
            nF = 0;
            continue;
        }
        if (capM < m) {           // accepted proposals only
            capM = m;
            for (uint64_t **p : {&bk, &bo, &uk, &uo, &nk, &no, &nk2, &no2})
                CK(grow((void **)p, capM * 8));
            for (int64_t **p : {&flag, &pos, &isnew, &npos}) CK(grow((void **)p, (capM + 1) * 8));
        }
        size_t b1 = 0, b2 = 0, b3 = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, b1, ak, bk, ao, bo, (int)m, 0, 64, s));
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, b2, flag, pos, m + 1, s));
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, b3, no, no2, nk, nk2, (int)m, 0, 64, s));
        CK(need_tmp(std::max(b1, std::max(b2, b3))));
        size_t tb = tmp_bytes;
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, ak, bk, ao, bo, (int)m, 0, 64, s));
        hipLaunchKernelGGL(k_bfs_heads, dim3((unsigned)((m + 1 + 255) / 256)), dim3(256), 0, s, m, bk,
                           flag);
        tb = tmp_bytes;
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, tb, flag, pos, m + 1, s));
        int64_t nu = 0;
        CK(hipMemcpyAsync(&nu, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        hipLaunchKernelGGL(k_bfs_unique, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, bk, bo,
                           pos, set, smask, uk, uo, isnew);
        CK(hipStreamSynchronize(s));
        // new states, in order of first occurrence
        CK(hipMemsetAsync(isnew + nu, 0, sizeof(int64_t), s));
        tb = tmp_bytes;
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, tb, isnew, npos, nu + 1, s));
        int64_t nn = 0;
        CK(hipMemcpyAsync(&nn, npos + nu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        hipLaunchKernelGGL(k_bfs_compact_new, dim3((unsigned)((nu + 255) / 256)), dim3(256), 0, s, nu,
                           uk, uo, isnew, npos, nk, no);
        CK(hipStreamSynchronize(s));
        if (nn > 0) {
            tb = tmp_bytes;
            CK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, no, no2, nk, nk2, (int)nn, 0, 64, s));
            const int64_t take = std::min<int64_t>(nn, nf - nS);
            hipLaunchKernelGGL(k_set_insert, dim3((unsigned)((take + 255) / 256)), dim3(256), 0, s,
                               take, nk2, set, smask, keys_dev, nS);
            CK(hipGetLastError());
            nS += take;
        }
        // next frontier: every accepted state once (sorted by key)
        if (capF < nu) {
            capF = nu;
            CK(grow((void **)&F, capF * 8));
        }
        CK(hipMemcpyAsync(F, uk, nu * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        nF = nu;
        CK(hipStreamSynchronize(s));
    }
    // output sorted
    {
        uint64_t *srt = nullptr;
        CK(dmalloc((void **)&srt, nS * sizeof(uint64_t), al));
        size_t b = 0;
        CK(hipcub::DeviceRadixSort::SortKeys(nullptr, b, keys_dev, srt, (int)nS, 0, 64, s));
        CK(need_tmp(b));
        b = tmp_bytes;
        CK(hipcub::DeviceRadixSort::SortKeys(tmp, b, keys_dev, srt, (int)nS, 0, 64, s));
        CK(hipMemcpyAsync(keys_dev, srt, nS * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        CK(hipStreamSynchronize(s));
        (void)dfree(srt, al);
    }
    *n_out = nS;
    if (steps_out) *steps_out = step;
    cleanup();
#undef CK
    return MCD_OK;
}

static int build_full(const mcd_model *model, const mcd_basis_cfg *cfg, uint64_t *keys_dev,
                      int64_t cap, int64_t *n_out, mcd_ws *ws, hipStream_t s) {
    const Alloc al{ws};
    Binom hb;
    fill_binom(hb);
    const int n = model->n_orb;
    const uint64_t nd_states = hb.c[n][cfg->n_dn];
    const uint64_t total = hb.c[n][cfg->n_up] * nd_states;
    *n_out = (int64_t)total;
    MCD_REQUIRE((int64_t)total <= cap, MCD_E_CAPACITY, "sector has %llu states, cap is %lld",
                (unsigned long long)total, (long long)cap);
    Binom *db = nullptr;
    MCD_HIP(dmalloc((void **)&db, sizeof(Binom), al));
    MCD_HIP(hipMemcpyAsync(db, &hb, sizeof(Binom), hipMemcpyHostToDevice, s));
    if (total)
        hipLaunchKernelGGL(k_enumerate, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                           total, nd_states, n, cfg->n_up, cfg->n_dn, db, keys_dev);
    MCD_HIP(hipGetLastError());
    MCD_HIP(hipStreamSynchronize(s));
    MCD_HIP(dfree(db, al));
    return MCD_OK;
}

static int build_chain(const mcd_model *model, const mcd_basis_cfg *cfg, uint64_t *keys_dev,
                       int64_t cap, int64_t *n_out, int64_t *steps_out, mcd_ws *ws,
                       hipStream_t s) {
    const Alloc al{ws};
    const uint64_t lim = model->n_orb >= 32 ? 0xffffffffull : ((1ull << model->n_orb) - 1ull);
    const uint64_t su = cfg->start_key >> 32, sd = cfg->start_key & 0xffffffffull;
    MCD_REQUIRE((su & ~lim) == 0 && (sd & ~lim) == 0 && __builtin_popcountll(su) == cfg->n_up &&
                    __builtin_popcountll(sd) == cfg->n_dn,
                MCD_E_SECTOR, "start key is not in the (%d, %d) sector", cfg->n_up, cfg->n_dn);
    MCD_REQUIRE(cfg->n_f >= 0 && cfg->burn_in >= 0 && cfg->max_steps >= 0, MCD_E_INVALID,
                "negative n_f, burn_in or max_steps");
    MCD_REQUIRE(model->n_bonds >= 1, MCD_E_INVALID, "a chain needs at least one bond");
    ChainWalker w;
    w.m = model;
    for (int b = 0; b < model->n_bonds; b++) {
        w.lo.push_back(std::min(model->bond_i[b], model->bond_j[b]));
        w.hi.push_back(std::max(model->bond_i[b], model->bond_j[b]));
    }
    w.up = su;
    w.dn = sd;
    w.rng.s = cfg->seed;
    w.beta = cfg->beta_s;
    w.burn_in = cfg->burn_in;

    const int64_t chunk = int64_t(1) << 24;
    uint64_t tcap = 1024;
    while (tcap < (uint64_t)(2 * (cfg->n_f + chunk))) tcap <<= 1;
    VisitSlot *tab = nullptr;
    uint64_t *d_ek = nullptr, *d_es = nullptr;
    unsigned long long *d_cnt = nullptr;
    uint64_t *d_steps = nullptr, *d_keys = nullptr, *d_steps2 = nullptr, *d_keys2 = nullptr;
    void *tmp = nullptr;
    auto cleanup = [&]() {
        for (void *p : {(void *)tab, (void *)d_ek, (void *)d_es, (void *)d_cnt, (void *)d_steps,
                        (void *)d_keys, (void *)d_steps2, (void *)d_keys2, tmp})
            if (p) (void)dfree(p, al);
    };
#define CK(expr)                                                                    \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));               \
            cleanup();                                                              \
            return hip_status(e_);                                                  \
        }                                                                           \
    } while (0)
    CK(dmalloc((void **)&tab, tcap * sizeof(VisitSlot), al));
    CK(hipMemsetAsync(tab, 0xff, tcap * sizeof(VisitSlot), s));
    CK(dmalloc((void **)&d_ek, chunk * sizeof(uint64_t), al));
    CK(dmalloc((void **)&d_es, chunk * sizeof(uint64_t), al));
    CK(dmalloc((void **)&d_cnt, 2 * sizeof(unsigned long long), al));
    CK(hipMemsetAsync(d_cnt, 0, 2 * sizeof(unsigned long long), s));
    std::vector<uint64_t> ek, es;
    ek.reserve(chunk);
    es.reserve(chunk);
    unsigned long long distinct = 0;
    while (w.step < cfg->max_steps && (int64_t)distinct < cfg->n_f) {
        ek.clear();
        es.clear();
        w.run(std::min<int64_t>(chunk, cfg->max_steps - w.step), ek, es);
        const int64_t m = (int64_t)ek.size();
        if (m) {
            CK(hipMemcpyAsync(d_ek, ek.data(), m * sizeof(uint64_t), hipMemcpyHostToDevice, s));
            CK(hipMemcpyAsync(d_es, es.data(), m * sizeof(uint64_t), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_visit_insert, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                               m, d_ek, d_es, tab, tcap - 1, d_cnt);
            CK(hipGetLastError());
        }
        CK(hipMemcpyAsync(&distinct, d_cnt, sizeof(distinct), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
    }
    const int64_t D = (int64_t)distinct;
    const int64_t nf = std::min<int64_t>(D, cfg->n_f);
    *n_out = nf;
    if (nf > cap) {
        cleanup();
        set_error("chain basis has %lld states, cap is %lld", (long long)nf, (long long)cap);
        return MCD_E_CAPACITY;
    }
    int64_t steps_done = w.step;
    if (D > 0) {
        CK(dmalloc((void **)&d_steps, D * sizeof(uint64_t), al));
        CK(dmalloc((void **)&d_keys, D * sizeof(uint64_t), al));
        CK(dmalloc((void **)&d_steps2, D * sizeof(uint64_t), al));
        CK(dmalloc((void **)&d_keys2, D * sizeof(uint64_t), al));
        hipLaunchKernelGGL(k_visit_compact, dim3((unsigned)((tcap + 255) / 256)), dim3(256), 0, s,
                           tcap, tab, d_steps, d_keys, d_cnt + 1);
        CK(hipGetLastError());
        size_t tb1 = 0, tb2 = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb1, d_steps, d_steps2, d_keys, d_keys2,
                                              (int)D, 0, 64, s));
        CK(hipcub::DeviceRadixSort::SortKeys(nullptr, tb2, d_keys2, keys_dev, (int)nf, 0, 64, s));
        const size_t tb = std::max(tb1, tb2);
        CK(dmalloc((void **)&tmp, tb, al));
        size_t t1 = tb;
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, t1, d_steps, d_steps2, d_keys, d_keys2, (int)D,
                                              0, 64, s));
        if ((int64_t)distinct >= cfg->n_f && nf > 0) {
            uint64_t last = 0;
            CK(hipMemcpyAsync(&last, d_steps2 + (nf - 1), sizeof(uint64_t), hipMemcpyDeviceToHost,
                              s));
            CK(hipStreamSynchronize(s));
            steps_done = (int64_t)last;
        }
        size_t t2 = tb;
        if (nf > 0)
            CK(hipcub::DeviceRadixSort::SortKeys(tmp, t2, d_keys2, keys_dev, (int)nf, 0, 64, s));
        CK(hipStreamSynchronize(s));
    }
    if (steps_out) *steps_out = steps_done;
    cleanup();
#undef CK
    return MCD_OK;
}

}  // namespace mcd

using namespace mcd;

extern "C" int mcd_basis_build(const mcd_model *model, const mcd_basis_cfg *cfg,
                               uint64_t *keys_dev, int64_t cap, int64_t *n_out,
                               int64_t *steps_out, mcd_ws *ws, void *stream) {
    MCD_REQUIRE(model && cfg && n_out, MCD_E_INVALID, "model, cfg or n_out is NULL");
    HostModel hm;
    MCD_TRY(prepare_model(model, &hm));
    MCD_REQUIRE(cfg->n_up >= 0 && cfg->n_dn >= 0 && cfg->n_up <= model->n_orb &&
                    cfg->n_dn <= model->n_orb,
                MCD_E_SECTOR, "sector (%d, %d) impossible with %d orbitals", cfg->n_up, cfg->n_dn,
                model->n_orb);
    MCD_REQUIRE(cap == 0 || keys_dev != nullptr, MCD_E_INVALID, "keys_dev is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (steps_out) *steps_out = 0;
    if (cfg->mode == MCD_BASIS_FULL) return build_full(model, cfg, keys_dev, cap, n_out, ws, s);
    if (cfg->mode == MCD_BASIS_CHAIN)
        return build_chain(model, cfg, keys_dev, cap, n_out, steps_out, ws, s);
    if (cfg->mode == MCD_BASIS_STEPS)
        return build_bfs(model, cfg, keys_dev, cap, n_out, steps_out, ws, s);
    set_error("basis mode %d unknown", cfg->mode);
    return MCD_E_INVALID;
}
