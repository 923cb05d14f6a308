// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include <string.h>

#include <mutex>

#include "mcd.h"
#include "mcd_wsalloc.h"

namespace mcd {

void set_error(const char *fmt, ...);

#define MCD_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            const int st_ = ::mcd::hip_status(e_);                                     \
            if (st_ == MCD_E_WORKSPACE)                                                \
                ::mcd::set_error("%s: workspace too small (%s:%d)", #expr, __FILE__,   \
                                 __LINE__);                                            \
            else                                                                       \
                ::mcd::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),\
                                 __FILE__, __LINE__);                                  \
            return st_;                                                                \
        }                                                                              \
    } while (0)

#define MCD_TRY(expr)                    \
    do {                                 \
        int rc_ = (expr);                \
        if (rc_ < 0) return rc_;         \
    } while (0)

#define MCD_REQUIRE(cond, code, ...)           \
    do {                                       \
        if (!(cond)) {                         \
            ::mcd::set_error(__VA_ARGS__);     \
            return (code);                     \
        }                                      \
    } while (0)

constexpr uint64_t kEmpty = ~0ull;           // hash sentinel, never a valid key
// Packed CSR word: column (col_bits) | amplitude class (31 - col_bits bits)
// | sign (bit 31).  col_bits = 31 - ceil(log2(classes)) is chosen per model,
// so one |t| allows 2^31 rows, two 2^30, ..., 32 classes 2^26.
constexpr int kMaxClasses = 32;              // packed CSR: distinct |t| values
constexpr int kStreamNnzMax = 4096;          // LDS products per stream block
constexpr int kStreamNnzSmall = 1024;        // ... of the small-block stream variant
constexpr int kBlockWordsLarge = 8192;      // column words of a large one-pass block-product tile
constexpr int kMergeBS = 256;                // merge-path SpMV: threads per workgroup
constexpr int kMergeDepth = 8;               // nonzeros per thread per chunk
constexpr int kMergeK = kMergeBS * kMergeDepth;  // path items (nonzeros + 9 per row) per chunk
constexpr int kMergeRowCost = 9;             // so a chunk ends < kMergeBS rows

enum {
    KERNEL_STREAM = 1,
    KERNEL_MERGE = 2,
    KERNEL_STREAM_XCD = 3,
    KERNEL_ROWCHUNK = 4,
    KERNEL_STREAM_S = 5,       // stream with <= kStreamNnzSmall products per block
    KERNEL_STREAM_S_XCD = 6,   // ... in XCD-major order
    KERNEL_GROUPED = 7,        // grouped entry order (coalesced up-hop gathers)
    KERNEL_GROUPED_XCD = 8,    // ... in XCD-major order
    KERNEL_LAST = 8
};
// Grouped one-vector layout: row blocks of <= kGroupedRows rows and
// <= kGroupedNnz nonzeros; <= kGroupedMaxGroups up-hop groups per block.
constexpr int kGroupedNnz = 3072;
constexpr int kGroupedRows = 256;
constexpr int kGroupedMaxGroups = 128;
constexpr int kNumXcd = 8;                   // gfx950: workgroups are dealt round-robin to 8 XCDs

// A pointer into global memory as such: loads and stores through it are
// global ones even where the pointer came from memory (a run table) and the
// compiler would otherwise use flat accesses, which wait together with LDS.
template <typename T>
using GPtr = __attribute__((address_space(1))) T *;

// One hopping bond with i < j, prepared for bit arithmetic.
struct DevBond {
    uint32_t mask;      // (1 << i) | (1 << j)
    uint32_t between;   // bits strictly between i and j
    double t;           // amplitude t_ij (duplicates merged)
    uint32_t cls;       // index of |t| in vtab
    uint32_t neg;       // 1 if t < 0
};

// Model in device memory (read-only in kernels).
struct DevModel {
    int n_orb;
    int n_bonds;
    int n_classes;
    uint32_t col_bits;          // packed CSR column bits
    uint32_t col_mask;          // (1 << col_bits) - 1
    double U[MCD_MAX_ORB];
    double eps[MCD_MAX_ORB];
    double vtab[kMaxClasses];   // |t| per class
    DevBond bonds[MCD_MAX_BONDS];
};

// Device memory.  The library allocates none of its own: every buffer is a
// piece of a caller-owned workspace (mcd_ws, a device buffer the caller hands
// over, e.g. a torch tensor), taken and released through Alloc.  Pieces are
// 256-byte aligned.  Work that uses a workspace is enqueued on one stream (the
// caller's), so a piece released on the host and taken again by a later call
// is only touched by kernels enqueued after the earlier ones: reuse is ordered
// by the stream, with no events and no device synchronisation.
struct Alloc {
    mcd_ws *ws = nullptr;
};
hipError_t dmalloc(void **p, size_t bytes, const Alloc &a);   // hipErrorOutOfMemory: ws full
hipError_t dfree(void *p, const Alloc &a);                    // NULL is ignored
// MCD status of a failed HIP call or allocation: MCD_E_WORKSPACE when the
// workspace ran out (dmalloc's hipErrorOutOfMemory), else MCD_E_HIP.
int hip_status(hipError_t e);
// Marks a piece of floating-point data just taken from a.ws: with the
// workspace's MCD_WS_POISON flag it is filled with all-ones bytes (NaN) on
// stream s, so reads before the first write show up in the results; a no-op
// otherwise.
hipError_t poison_fp(void *p, size_t bytes, const Alloc &a, hipStream_t s);

// Pieces taken together and released together (reverse order of taking):
// every buffer of a short-lived step (a band run and its operator) in one
// place.  One owner thread.
struct Arena {
    Alloc al;
    std::vector<void *> pieces;
    explicit Arena(mcd_ws *ws) { al.ws = ws; }
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    ~Arena() { release(); }
    hipError_t get(void **p, size_t bytes) {
        const hipError_t e = dmalloc(p, bytes, al);
        if (e == hipSuccess) pieces.push_back(*p);
        return e;
    }
    void release() {
        for (auto it = pieces.rbegin(); it != pieces.rend(); ++it) (void)dfree(*it, al);
        pieces.clear();
    }
};

struct HashSlot {
    uint64_t key;
    int64_t val;
};

// Host mirror of the model: bonds merged (same unordered pair -> summed t).
struct HostModel {
    DevModel dm;
    bool ok_classes;     // <= kMaxClasses distinct |t|
};

int prepare_model(const mcd_model *m, HostModel *hm);

}  // namespace mcd

// A caller-owned workspace: the caller's device buffer [base, base + size)
// and the host bookkeeping of the pieces taken from it.
struct mcd_ws {
    char *base;
    mcd::WsAlloc a;
    std::mutex mu;
    int debug = 0;   // MCD_WS_POISON
    mcd_ws(void *b, size_t bytes) : base((char *)b), a(bytes) {}
};

struct mcd_op {
    int device;
    int64_t n;
    int32_t storage;
    int32_t rows_per_block;    // stream kernel: rows per block (<= kStreamNnzMax nonzeros)
    int32_t rows_per_block_s;  // small-block stream kernel (<= kStreamNnzSmall nonzeros)
    int32_t rows_per_block_l;  // rows per block with <= kBlockWordsLarge nonzeros
    int32_t group_chunk;       // row-parallel products: packed words per chunk (4, 8 or 16)
    int64_t nnz;
    int64_t device_bytes;
    double build_ms;
    mcd::HostModel hm;
    mcd::DevModel *d_model;
    uint64_t *d_keys;
    double *d_diag;
    mcd::HashSlot *d_hash;
    uint64_t hash_mask;
    int64_t *d_rowptr;
    uint32_t *d_colw;
    // scratch for grid reductions
    double *d_partials;        // [max blocks]
    unsigned int *d_counter;   // last-block counters [8]
    double *d_scalars;         // [64]
    int64_t max_partials;
    // merge-path SpMV: chunk split points and carries
    int32_t kernel;            // KERNEL_STREAM or KERNEL_MERGE (one-vector CSR)
    int32_t merge_grid;        // persistent workgroups
    int64_t nchunks;
    int64_t *d_split_i, *d_split_j;   // [nchunks + 1]
    double *d_carry;                  // [nchunks]
    int64_t *d_carry_row;             // [nchunks]
    double tune_ms[mcd::KERNEL_LAST + 1];  // measured per-apply time per kernel
    // grouped one-vector layout (g_nblocks = 0: not built or not applicable)
    int64_t g_nblocks;
    int64_t g_ngroups;
    int64_t *d_gbs;                   // [g_nblocks + 1] first row of each block
    int64_t *d_goff;                  // [g_nblocks + 1] first group of each block
    int64_t *d_gbe;                   // [g_nblocks + 1] first entry of each block
    uint32_t *d_gtab;                 // [g_ngroups + 1] column | class << 28 | sign << 31
    uint32_t *d_gw;                   // [nnz] entry words in grouped order
    mcd::Alloc alloc;                 // the workspace the operator's buffers come from
};

namespace mcd {

// Operator internals used by the solvers (defined in mcd_op.hip).
// y = sx * H (x) for one double vector, sx read on the device (sx_mode 0:
// *sx_dev, 1: 1/sqrt(*sx_dev), sx_dev == nullptr: 1); when dot_out !=
// nullptr the scalar sum_r (sx x_r) y_r is written to *dot_out (device).
int apply_f64_fused(const mcd_op *op, const double *x, double *y, const double *sx_dev,
                    int sx_mode, double *dot_out, hipStream_t s);
// The same for a float32 or float64 vector (float accumulation for float32;
// the scale and the dot are float64).
template <typename T>
int apply_fused(const mcd_op *op, const T *x, T *y, const double *sx_dev, int sx_mode,
                double *dot_out, hipStream_t s);
// y *= sx and optional dot as above (used after an on-the-fly apply).
template <typename T>
int scale_dot(const mcd_op *op, T *y, const T *x, const double *sx_dev, int sx_mode,
              double *dot_out, hipStream_t s);
int apply_any(const mcd_op *op, int dtype, int nvec, const void *x, void *y, hipStream_t s);

// Grouped one-vector layout (mcd_grouped.hip).  build_grouped leaves
// g_nblocks = 0 when the basis does not fit the layout (short up-string
// segments, too many groups per block, offsets out of range); only HIP
// errors are returned as errors.  grouped_one launches the product (same
// contract as the other one-vector kernels; partials per workgroup when
// `partials` != nullptr, *grid = number of workgroups).
int build_grouped(mcd_op *op, hipStream_t s);
void grouped_plan(WsAlloc &w, int64_t n, int64_t nnz);
template <typename T>
int grouped_one(const mcd_op *op, bool xcd, const T *x, T *y, const double *sx_dev, int sx_mode,
                double *partials, int64_t *grid, hipStream_t s);


// Operator construction (mcd_op_create with tune = true); tune = false keeps
// the default one-vector kernel (for operators used with block products).
// Every buffer comes from `ws` and goes back to it in mcd_op_destroy.
int op_create(const mcd_model *model, const uint64_t *keys_dev, int64_t n, int32_t storage,
              int32_t validate, bool tune, mcd_ws *ws, void *stream, mcd_op **out);
// Workspace bytes op_create takes from an empty workspace (stages: 1 index,
// 2 up to the nonzero count, 3 all but the grouped layout, 4 with the largest
// grouped layout).
size_t op_plan(int64_t n, bool csr, int64_t nnz, bool tune, bool validate, int stages,
               int n_bonds);

// Deterministic dot product a . b into *out_dev (mcd_lanczos.hip).
int dev_dot(const mcd_op *op, const double *a, const double *b, int64_t n, double *out_dev,
            hipStream_t s);

}  // namespace mcd
