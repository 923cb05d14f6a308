// Parameter derivatives of H~ contracted with two vectors:
//   <a| dH~/dt_b |b>   for every listed bond b (the hop operator of the pair,
//                      both spins, both directions, discarded outside F~),
//   <a| dH~/dU_i |b>   = sum_r a_r b_r n_{i up} n_{i dn}(r),
//   <a| dH~/deps_i |b> = sum_r a_r b_r (n_{i up} + n_{i dn})(r).
// With a = b = |Omega> these are the Hellmann-Feynman derivatives dE0/dtheta
// of the ground-state energy (Eq. hubbard_model with theta = t_ij, U_i, eps_i).
// One pass over the rows; each workgroup keeps one partial per parameter and
// the partials are added in index order (deterministic).
#include <algorithm>
#include <mutex>
#include <vector>

#include "mcd_hash.h"
#include "mcd_internal.h"
#include "mcd_reduce.h"

namespace mcd {

static constexpr int GBS = 256;

static constexpr int kMaxContractBlocks = 2048;
static constexpr int kMaxParams = MCD_MAX_BONDS + 2 * MCD_MAX_ORB;

// part[p * gridDim.x + block] for p in [0, NB + 2 n_orb): merged bonds, U_i,
// eps_i.  Workgroup b takes the row tiles b, b + G, ... (G = gridDim.x) and
// adds each tile's workgroup sum to its per-parameter total in tile order.
__global__ __launch_bounds__(GBS) void k_contract(int64_t n, const uint64_t *__restrict__ keys,
                                                  const DevModel *__restrict__ m,
                                                  const HashSlot *__restrict__ h, uint64_t hmask,
                                                  const double *__restrict__ a,
                                                  const double *__restrict__ b,
                                                  double *__restrict__ part) {
    __shared__ double tot[kMaxParams];
    const int nb = m->n_bonds, no = m->n_orb, np = nb + 2 * no;
    for (int i = threadIdx.x; i < np; i += GBS) tot[i] = 0.0;
    __syncthreads();
    for (int64_t tile = blockIdx.x; tile * GBS < n; tile += gridDim.x) {
        const int64_t r = tile * GBS + threadIdx.x;
        const bool own = r < n;
        const uint64_t key = own ? keys[r] : 0ull;
        const double ar = own ? a[r] : 0.0;
        const double br = own ? b[r] : 0.0;
        const uint32_t up = (uint32_t)(key >> 32), dn = (uint32_t)key;
        for (int q = 0; q < nb; q++) {
            double c = 0.0;
            if (own) {
                const uint32_t mask = m->bonds[q].mask, between = m->bonds[q].between;
                if (__popc(up & mask) == 1) {
                    const int64_t col = hash_find(h, hmask, key ^ ((uint64_t)mask << 32));
                    if (col >= 0) c += (__popc(up & between) & 1) ? -b[col] : b[col];
                }
                if (__popc(dn & mask) == 1) {
                    const int64_t col = hash_find(h, hmask, key ^ (uint64_t)mask);
                    if (col >= 0) c += (__popc(dn & between) & 1) ? -b[col] : b[col];
                }
                c *= ar;
            }
            c = block_sum<GBS>(c);
            if (threadIdx.x == 0) tot[q] += c;
        }
        for (int i = 0; i < no; i++) {
            const double nu = (double)((up >> i) & 1u), nd = (double)((dn >> i) & 1u);
            const double ab = ar * br;
            const double cu = block_sum<GBS>(ab * (nu * nd));
            if (threadIdx.x == 0) tot[nb + i] += cu;
            const double ce = block_sum<GBS>(ab * (nu + nd));
            if (threadIdx.x == 0) tot[nb + no + i] += ce;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np; i += GBS) part[(int64_t)i * gridDim.x + blockIdx.x] = tot[i];
}

__global__ __launch_bounds__(256) void k_contract_reduce(int np, int64_t nblk,
                                                         const double *__restrict__ part,
                                                         double *__restrict__ out) {
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= np) return;
    double s = 0.0;
    for (int64_t c = lane; c < nblk; c += 64) s += part[(int64_t)p * nblk + c];
    s = wave_sum(s);
    if (lane == 0) out[p] = s;
}

static int contract_blocks(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + GBS - 1) / GBS, kMaxContractBlocks));
}

// The contraction with partials in `part` ([np][nblk] + np doubles) and the
// host-side mapping of merged bonds back to listed bonds.
static int contract_into(const mcd_op *op, const mcd_model *model, const double *a_dev,
                         const double *b_dev, double *part, double *d_t, double *d_U,
                         double *d_eps, hipStream_t s) {
    const int nb = op->hm.dm.n_bonds, no = op->hm.dm.n_orb;
    const int np = nb + 2 * no;
    const int nblk = contract_blocks(op->n);
    double *out = part + (size_t)np * nblk;
    hipLaunchKernelGGL(k_contract, dim3((unsigned)nblk), dim3(GBS), 0, s, op->n, op->d_keys,
                       op->d_model, op->d_hash, op->hash_mask, a_dev, b_dev, part);
    hipLaunchKernelGGL(k_contract_reduce, dim3((unsigned)((np + 3) / 4)), dim3(256), 0, s, np,
                       (int64_t)nblk, part, out);
    MCD_HIP(hipGetLastError());
    double h[kMaxParams];   // np <= kMaxParams (merged bonds <= listed bonds)
    MCD_HIP(hipMemcpyAsync(h, out, np * sizeof(double), hipMemcpyDeviceToHost, s));
    MCD_HIP(hipStreamSynchronize(s));
    // listed bond -> merged pair (bonds listed twice share the pair's derivative)
    if (d_t) {
        for (int q = 0; q < model->n_bonds; q++) {
            const int i = std::min(model->bond_i[q], model->bond_j[q]);
            const int j = std::max(model->bond_i[q], model->bond_j[q]);
            const uint32_t mask = (1u << i) | (1u << j);
            double v = 0.0;
            for (int mb = 0; mb < nb; mb++)
                if (op->hm.dm.bonds[mb].mask == mask) v = h[mb];
            d_t[q] = v;
        }
    }
    for (int i = 0; i < no; i++) {
        if (d_U) d_U[i] = h[nb + i];
        if (d_eps) d_eps[i] = h[nb + no + i];
    }
    return MCD_OK;
}

static size_t contract_scratch_bytes(const mcd_op *op) {
    const int np = op->hm.dm.n_bonds + 2 * op->hm.dm.n_orb;
    return ((size_t)np * contract_blocks(op->n) + np) * sizeof(double);
}

// Scratch of the allocation-free contraction: the workgroup partials of the
// largest parameter count at the largest grid, and the reduced values
// (9.4 MB per device, held until the process ends).  Host code never passes
// `scratch` itself to a kernel: its address on a device is looked up once
// per device (hipGetSymbolAddress, with that device current) and kept.
constexpr size_t kNoAllocDoubles = (size_t)kMaxParams * kMaxContractBlocks + kMaxParams;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[64] = {};

static int scratch_address(int dev, double **out) {
    MCD_REQUIRE(dev >= 0 && dev < 64, MCD_E_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return MCD_E_HIP;
        }
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MCD_OK;
}

}  // namespace mcd

using namespace mcd;

extern "C" int mcd_hamiltonian_contract(const mcd_op *op, const mcd_model *model,
                                        const double *a_dev, const double *b_dev, double *d_t,
                                        double *d_U, double *d_eps, mcd_ws *ws, void *stream) {
    MCD_REQUIRE(op && model && a_dev && b_dev, MCD_E_INVALID, "op, model, a, b required");
    MCD_REQUIRE(model->n_orb == op->hm.dm.n_orb, MCD_E_INVALID,
                "model has %d orbitals, operator %d", model->n_orb, op->hm.dm.n_orb);
    hipStream_t s = (hipStream_t)stream;
    const Alloc al{ws};
    double *part = nullptr;
    MCD_HIP(dmalloc((void **)&part, contract_scratch_bytes(op), al));
    if (poison_fp(part, contract_scratch_bytes(op), al, s) != hipSuccess) {
        (void)dfree(part, al);
        set_error("contract: workspace fill failed");
        return MCD_E_HIP;
    }
    const int rc = contract_into(op, model, a_dev, b_dev, part, d_t, d_U, d_eps, s);
    (void)hipStreamSynchronize(s);
    (void)dfree(part, al);
    return rc;
}

extern "C" int mcd_hamiltonian_contract_noalloc(const mcd_op *op, const mcd_model *model,
                                                const double *a_dev, const double *b_dev,
                                                double *d_t, double *d_U, double *d_eps,
                                                void *stream) {
    MCD_REQUIRE(op && model && a_dev && b_dev, MCD_E_INVALID, "op, model, a, b required");
    MCD_REQUIRE(model->n_orb == op->hm.dm.n_orb, MCD_E_INVALID,
                "model has %d orbitals, operator %d", model->n_orb, op->hm.dm.n_orb);
    MCD_REQUIRE(contract_scratch_bytes(op) <= kNoAllocDoubles * sizeof(double), MCD_E_CAPACITY,
                "contraction needs %zu bytes of scratch, the fixed scratch holds %zu",
                contract_scratch_bytes(op), kNoAllocDoubles * sizeof(double));
    int dev = 0;
    MCD_HIP(hipGetDevice(&dev));
    double *part = nullptr;
    MCD_TRY(scratch_address(dev, &part));
    // every partial and output the reduction reads is written by this call's
    // kernels first (k_contract writes all np x nblk partials)
    return contract_into(op, model, a_dev, b_dev, part, d_t, d_U, d_eps, (hipStream_t)stream);
}
