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

int hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? MCD_E_WORKSPACE : MCD_E_HIP; }

hipError_t dmalloc(void **p, size_t bytes, const Alloc &a) {
    *p = nullptr;
    if (a.ws == nullptr) return hipErrorOutOfMemory;   // no workspace: nothing to take
    std::lock_guard<std::mutex> lock(a.ws->mu);
    const size_t off = a.ws->a.alloc(bytes);
    if (off == WsAlloc::kFail) return hipErrorOutOfMemory;
    *p = a.ws->base + off;
    return hipSuccess;
}

hipError_t dfree(void *p, const Alloc &a) {
    if (p == nullptr || a.ws == nullptr) return hipSuccess;
    std::lock_guard<std::mutex> lock(a.ws->mu);
    const char *c = (const char *)p;
    if (c < a.ws->base || !a.ws->a.release((size_t)(c - a.ws->base))) return hipErrorInvalidValue;
    return hipSuccess;
}

// All-ones 16-byte words over a piece (pieces are whole 256-byte units).
__global__ __launch_bounds__(256) void k_poison(uint4 *p, int64_t words) {
    const uint4 v = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

hipError_t poison_fp(void *p, size_t bytes, const Alloc &a, hipStream_t s) {
    if (p == nullptr || a.ws == nullptr || !(a.ws->debug & MCD_WS_POISON)) return hipSuccess;
    const int64_t words = (int64_t)(WsAlloc::round(bytes) / 16);
    const unsigned grid = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_poison, dim3(grid), dim3(256), 0, s, (uint4 *)p, words);
    return hipGetLastError();
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

extern "C" int mcd_ws_create(void *base_dev, size_t bytes, mcd_ws **out) {
    MCD_REQUIRE(out != nullptr, MCD_E_INVALID, "out is NULL");
    *out = nullptr;
    MCD_REQUIRE(base_dev != nullptr || bytes == 0, MCD_E_INVALID, "base is NULL");
    MCD_REQUIRE(((uintptr_t)base_dev & 255u) == 0, MCD_E_INVALID,
                "workspace base must be 256-byte aligned");
    mcd_ws *w = new mcd_ws(base_dev, bytes);
    *out = w;
    return MCD_OK;
}

extern "C" void mcd_ws_destroy(mcd_ws *ws) { delete ws; }

extern "C" int mcd_ws_stats(const mcd_ws *ws, size_t *size, size_t *in_use, size_t *high_water,
                            size_t *need) {
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "ws is NULL");
    std::lock_guard<std::mutex> lock(const_cast<mcd_ws *>(ws)->mu);
    if (size) *size = ws->a.size();
    if (in_use) *in_use = ws->a.in_use();
    if (high_water) *high_water = ws->a.high_water();
    if (need) *need = ws->a.need();
    return MCD_OK;
}

extern "C" int mcd_ws_set_debug(mcd_ws *ws, int32_t flags) {
    MCD_REQUIRE(ws != nullptr, MCD_E_INVALID, "ws is NULL");
    MCD_REQUIRE((flags & ~MCD_WS_POISON) == 0, MCD_E_INVALID, "unknown workspace flags 0x%x",
                (unsigned)flags);
    std::lock_guard<std::mutex> lock(ws->mu);
    ws->debug = flags;
    return MCD_OK;
}
extern "C" int mcd_version(void) { return 10000; }
