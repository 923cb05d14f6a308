// Error reporting and model preparation shared by the library.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "mcd_internal.h"

namespace mcd {

static thread_local char g_err[1024] = "";

namespace {
struct CachedChunk {
    char *p;
    size_t bytes;
    int dev;
    hipEvent_t ready;   // recorded on the releasing stream
};
std::mutex g_chunk_mu;
std::vector<CachedChunk> g_chunks;   // free chunks
size_t g_chunk_bytes = 0;            // bytes held by g_chunks
}  // namespace

hipError_t chunk_acquire(size_t bytes, hipStream_t s, void **out, size_t *got) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lock(g_chunk_mu);
        int best = -1;
        for (int i = 0; i < (int)g_chunks.size(); i++) {
            const CachedChunk &c = g_chunks[i];
            if (c.dev != dev || c.bytes < bytes || c.bytes > 2 * bytes + (size_t(64) << 20))
                continue;
            if (best < 0 || c.bytes < g_chunks[best].bytes) best = i;
        }
        if (best >= 0) {
            const CachedChunk c = g_chunks[best];
            g_chunks.erase(g_chunks.begin() + best);
            g_chunk_bytes -= c.bytes;
            e = hipStreamWaitEvent(s, c.ready, 0);
            (void)hipEventDestroy(c.ready);
            if (e != hipSuccess) {
                (void)hipFree(c.p);
                return e;
            }
            *out = c.p;
            *got = c.bytes;
            return hipSuccess;
        }
    }
    const size_t unit = size_t(64) << 20;
    const size_t sz = (std::max<size_t>(bytes, 1) + unit - 1) / unit * unit;
    e = hipMalloc(out, sz);
    if (e != hipSuccess) {
        // free this device's cached chunks once, then retry
        (void)hipGetLastError();
        std::vector<CachedChunk> mine;
        {
            std::lock_guard<std::mutex> lock(g_chunk_mu);
            for (auto it = g_chunks.begin(); it != g_chunks.end();) {
                if (it->dev == dev) {
                    mine.push_back(*it);
                    g_chunk_bytes -= it->bytes;
                    it = g_chunks.erase(it);
                } else {
                    ++it;
                }
            }
        }
        for (auto &c : mine) {
            (void)hipEventSynchronize(c.ready);
            (void)hipEventDestroy(c.ready);
            (void)hipFree(c.p);
        }
        e = hipMalloc(out, sz);
    }
    if (e == hipSuccess) *got = sz;
    return e;
}

void chunk_release(void *p, size_t bytes, hipStream_t s) {
    int dev = 0;
    hipEvent_t ev = nullptr;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess) {
        (void)hipStreamSynchronize(s);
        if (ev) (void)hipEventDestroy(ev);
        (void)hipFree(p);
        return;
    }
    {
        std::lock_guard<std::mutex> lock(g_chunk_mu);
        if (g_chunk_bytes + bytes <= kChunkCacheBytes) {
            g_chunks.push_back({(char *)p, bytes, dev, ev});
            g_chunk_bytes += bytes;
            return;
        }
    }
    (void)hipEventSynchronize(ev);
    (void)hipEventDestroy(ev);
    (void)hipFree(p);
}

void pool_keep_freed(int device) {
    static std::mutex mu;
    static bool done[64] = {};
    if (device < 0 || device >= 64) return;
    std::lock_guard<std::mutex> lock(mu);
    if (done[device]) return;
    done[device] = true;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess || pool == nullptr) return;
    uint64_t keep = kPoolKeepBytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
}

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

// Validate the model, merge bonds that join the same pair (their amplitudes
// add, as two listed terms of Eq. hubbard_model would) and assign each
// distinct |t| a class index for the packed CSR.
int prepare_model(const mcd_model *m, HostModel *hm) {
    MCD_REQUIRE(m != nullptr, MCD_E_INVALID, "model is NULL");
    MCD_REQUIRE(m->n_orb >= 1 && m->n_orb <= MCD_MAX_ORB, MCD_E_INVALID,
                "n_orb = %d outside 1..%d", m->n_orb, MCD_MAX_ORB);
    MCD_REQUIRE(m->n_bonds >= 0 && m->n_bonds <= MCD_MAX_BONDS, MCD_E_INVALID,
                "n_bonds = %d outside 0..%d", m->n_bonds, MCD_MAX_BONDS);
    MCD_REQUIRE(m->U && m->eps, MCD_E_INVALID, "U or eps is NULL");
    MCD_REQUIRE(m->n_bonds == 0 || (m->bond_i && m->bond_j && m->bond_t), MCD_E_INVALID,
                "bond arrays are NULL");
    DevModel &d = hm->dm;
    memset(&d, 0, sizeof(d));
    d.n_orb = m->n_orb;
    for (int i = 0; i < m->n_orb; i++) {
        d.U[i] = m->U[i];
        d.eps[i] = m->eps[i];
    }
    std::vector<std::pair<std::pair<int, int>, double>> merged;
    std::map<std::pair<int, int>, size_t> where;
    for (int b = 0; b < m->n_bonds; b++) {
        int i = m->bond_i[b], j = m->bond_j[b];
        MCD_REQUIRE(i >= 0 && j >= 0 && i < m->n_orb && j < m->n_orb && i != j, MCD_E_INVALID,
                    "bond %d joins (%d, %d): orbitals must differ and be < n_orb", b, i, j);
        std::pair<int, int> key(std::min(i, j), std::max(i, j));
        auto it = where.find(key);
        if (it == where.end()) {
            where[key] = merged.size();
            merged.push_back({key, m->bond_t[b]});
        } else {
            merged[it->second].second += m->bond_t[b];
        }
    }
    std::vector<double> classes;
    int nb = 0;
    hm->ok_classes = true;
    for (auto &e : merged) {
        // zero-amplitude pairs are kept: their elements are zero, but the
        // derivative of H with respect to their amplitude is not
        double t = e.second;
        int i = e.first.first, j = e.first.second;
        DevBond &b = d.bonds[nb++];
        b.mask = (1u << i) | (1u << j);
        b.between = (uint32_t)(((1ull << j) - 1ull) & ~((1ull << (i + 1)) - 1ull));
        b.t = t;
        b.neg = t < 0.0 ? 1u : 0u;
        double a = fabs(t);
        int c = -1;
        for (size_t k = 0; k < classes.size(); k++)
            if (classes[k] == a) c = (int)k;
        if (c < 0) {
            c = (int)classes.size();
            classes.push_back(a);
        }
        if (c >= kMaxClasses) {
            hm->ok_classes = false;
            c = 0;
        }
        b.cls = (uint32_t)c;
    }
    d.n_bonds = nb;
    d.n_classes = (int)std::min<size_t>(classes.size(), kMaxClasses);
    uint32_t cls_bits = 0;
    while ((1 << cls_bits) < d.n_classes) cls_bits++;
    d.col_bits = 31u - cls_bits;
    d.col_mask = (d.col_bits >= 32) ? 0xffffffffu : ((1u << d.col_bits) - 1u);
    for (int k = 0; k < d.n_classes; k++) d.vtab[k] = classes[k];
    return MCD_OK;
}

}  // namespace mcd

extern "C" const char *mcd_last_error(void) { return mcd::g_err; }
extern "C" int mcd_version(void) { return 10000; }
