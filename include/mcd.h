/* mcd.h -- C ABI of the MI355X (gfx950) Monte Carlo diagonalization library.
 *
 * Monte Carlo diagonalization (MCD) solves the Hubbard model in a truncated
 * Fock basis F~ of "important" states (Sec. Subspace of the ground state):
 * the Hamiltonian is restricted to F~ (Eq. h_matrix_projected), the ground
 * state is found with Lanczos (App. Lanczos), and the Green function with
 * band Lanczos on the excited subspaces F~+- (Eq. excited_subspace,
 * App. Band Lanczos, Eqs. green_qmatrix / q_matrix).  Every step applies H~
 * to vectors; states that H sends outside the basis are discarded (App.
 * Lanczos, last paragraph).  This library runs that product and the solvers
 * around it on one GPU.
 *
 * Conventions shared by every call
 * --------------------------------
 * Model.  H = sum_b sum_s t_b (c+_{i_b s} c_{j_b s} + h.c.)
 *           + sum_i U_i n_{i up} n_{i dn} + sum_{i s} eps_i n_{i s}
 *   (Eq. hubbard_model with -t on nearest-neighbour bonds and eps_i = -mu on
 *   lattice sites; per-orbital U_i and eps_i cover impurity + bath models).
 *   Bonds listed twice add up.  n_orb <= 32, n_bonds <= MCD_MAX_BONDS.
 * Fock state.  A uint64 key (up << 32) | down, orbital i <-> bit i of each
 *   spin string.  A basis is an array of keys sorted ascending and unique;
 *   the row/column index of a state is its position in that array.
 * Fermion signs.  Orbital order "all up orbitals, then all down": a hop
 *   c+_{i s} c_{j s} carries (-1)^(number of s-electrons strictly between i
 *   and j); c+_{i s} or c_{i s} carries (-1)^(electrons in orbitals ordered
 *   before (i, s)).
 * Memory.  Pointers named *_dev are device pointers on the current HIP
 *   device; all others are host pointers.  The library allocates no device
 *   memory: every device buffer it uses is a piece of a caller-owned
 *   workspace (mcd_ws, below) -- typically a torch tensor -- and device
 *   inputs and outputs belong to the caller.  An operator handle holds its
 *   copy of the keys, index, CSR and reduction scratch in the workspace it
 *   was created from until mcd_op_destroy; a solver call takes its scratch
 *   from the workspace it is given and returns it before it returns.  Size
 *   queries (mcd_op_workspace_size, mcd_lanczos_workspace_size,
 *   mcd_band_workspace_size) give the bytes a call needs from an empty
 *   workspace; a call whose workspace runs out returns MCD_E_WORKSPACE
 *   having released what it took, and mcd_ws_stats reports a size at which
 *   the failing request would have been served (the caller may grow its
 *   buffer to it and call again).
 * Streams.  `stream` is a hipStream_t (NULL = default stream).  Work is
 *   enqueued on it and nowhere else: the library creates no streams and no
 *   host threads that touch the GPU (the band calls' host-side dense work --
 *   continued fractions, per-frequency solves -- runs on a process-wide pool
 *   of up to 15 worker threads, created on first use, that never call HIP;
 *   and a band call pins a small host buffer, the ranks and T of its runs,
 *   for its asynchronous read-backs, freed before it returns).  Calls that
 *   return host values
 *   synchronise it first and say so.  All calls that use one workspace must
 *   be ordered on one stream (a released piece is reused by later work on
 *   that stream); calls on one operator from several host threads or streams
 *   at once race on its scratch buffers.
 * Errors.  Every call returns MCD_OK (0), a positive warning (the result is
 *   still written) or a negative error code; mcd_last_error() gives a
 *   message for the calling thread.  Nothing aborts or throws across the ABI.
 */
#ifndef MCD_H
#define MCD_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCD_MAX_ORB 32
#define MCD_MAX_BONDS 512

enum {
    MCD_OK = 0,
    MCD_NOCONV = 1,          /* warning: iteration cap reached before tol */
    MCD_E_INVALID = -1,      /* bad argument (null pointer, size, range) */
    MCD_E_SECTOR = -2,       /* key outside the sector, unsorted or duplicate */
    MCD_E_HIP = -3,          /* a HIP runtime call failed */
    MCD_E_CAPACITY = -4,     /* output buffer or format limit too small */
    MCD_E_WORKSPACE = -5,    /* the caller's workspace is too small (see mcd_ws_stats) */
    MCD_E_NUMERIC = -6,      /* a non-finite value (NaN / Inf) in an input or in the
                                recurrence coefficients read back from the device */
    MCD_E_BREAKDOWN = -7,    /* a solve met a degenerate or indefinite system */
};

enum { MCD_STORAGE_AUTO = 0, MCD_STORAGE_ON_THE_FLY = 1, MCD_STORAGE_CSR = 2 };
enum { MCD_F64 = 0, MCD_F32 = 1 };
enum { MCD_BASIS_FULL = 0, MCD_BASIS_CHAIN = 1, MCD_BASIS_STEPS = 2 };

typedef struct mcd_model {
    int32_t n_orb;            /* orbitals (sites), 1..32 */
    int32_t n_bonds;          /* 0..MCD_MAX_BONDS */
    const int32_t *bond_i;    /* [n_bonds] host */
    const int32_t *bond_j;    /* [n_bonds] host, bond_i != bond_j */
    const double *bond_t;     /* [n_bonds] host, amplitude t_ij */
    const double *U;          /* [n_orb] host, on-site repulsion */
    const double *eps;        /* [n_orb] host, orbital energy (includes -mu) */
} mcd_model;

typedef struct mcd_op mcd_op;
typedef struct mcd_ws mcd_ws;

const char *mcd_last_error(void);
int mcd_version(void);

/* ---------------------------------------------------------------------------
 * Workspace.  mcd_ws_create wraps a caller-owned device buffer of `bytes`
 * bytes at base_dev (256-byte aligned; e.g. a torch.uint8 tensor's
 * data_ptr()).  Only host bookkeeping is created: the buffer stays the
 * caller's and must outlive the handle and every operator or kept run made
 * from it.  Pieces are handed out first-fit, 256-byte aligned.
 * mcd_ws_stats: size, bytes in use, the most ever in use, and `need` -- after
 * a call returned MCD_E_WORKSPACE, a workspace size at which the failing
 * request would have been served (0 if none failed).  Any output may be
 * NULL.  mcd_ws_destroy frees the bookkeeping only (NULL is ignored).
 * ------------------------------------------------------------------------- */
int mcd_ws_create(void *base_dev, size_t bytes, mcd_ws **out);
void mcd_ws_destroy(mcd_ws *ws);
int mcd_ws_stats(const mcd_ws *ws, size_t *size, size_t *in_use, size_t *high_water,
                 size_t *need);

/* Debugging aid.  With MCD_WS_POISON set, every floating-point piece the
 * library takes from `ws` from then on (vectors, Krylov blocks, Gram
 * partials, coefficient and recurrence stores, reduction scratch) is filled
 * with all-ones bytes -- NaN in float32 and float64 -- by a kernel on the
 * taking call's stream, so any result that depends on a read of such a piece
 * before its first write comes out NaN (or differs from an unpoisoned call).
 * Index, key and counter pieces are left as they are.  Results of correct
 * code are bit for bit those without the flag; the fills cost time only.
 * flags = 0 turns it off.  MCD_E_INVALID for a NULL handle or unknown bits. */
#define MCD_WS_POISON 1
int mcd_ws_set_debug(mcd_ws *ws, int32_t flags);

/* ---------------------------------------------------------------------------
 * mcd_basis_build -- the truncated basis F~ (Sec. Subspace of the ground
 * state; Sec. Other sampling methods).
 *
 * mode MCD_BASIS_FULL: every state of the (n_up, n_dn) sector, sorted
 *   (the f = 1 case, Sec. Exact diagonalization); n_out = C(n,n_up)C(n,n_dn).
 * mode MCD_BASIS_CHAIN: the distinct states visited by a Metropolis chain
 *   that proposes one random hop per step (variant 2) and accepts it with the
 *   ratio of Boltzmann factors of the diagonal energy (variant 1, Eq.
 *   boltzmann_factor2) at inverse temperature beta_s.  Draws come from
 *   splitmix64(seed), two per step: r0 picks m = (hi32(r0) * 4 n_bonds) >> 32
 *   (bond m >> 2, spin (m >> 1) & 1 with 0 = up, direction m & 1 with 0 =
 *   i -> j); an impossible hop is a rejected step; dE = (eps[dst]-eps[src])
 *   + (U[dst] o[dst] - U[src] o[src]) (o = other-spin occupation) and the
 *   hop is taken iff dE <= 0 or (r1 >> 11) 2^-53 < exp(-beta_s dE).  After
 *   burn_in steps the state after every step is recorded; the basis is the
 *   first n_f distinct recorded states (or all of them if max_steps ends the
 *   chain first), sorted.  steps_out = steps the chain ran.
 *   The chain itself is sequential and runs on the host; recording,
 *   de-duplication, first-visit selection and sorting run on the GPU.
 * mode MCD_BASIS_STEPS: the paper's own sampler (Sec. Subspace of the ground
 *   state, the numbered "step" procedure, Eq. boltzmann_factor), entirely on
 *   the GPU.  F~ and the frontier start as {start_key}.  A step applies every
 *   hop h in [0, 4 n_bonds) (bond h >> 2, spin (h >> 1) & 1, direction h & 1)
 *   to every frontier state (ascending keys); a possible hop is accepted iff
 *   u < exp(-beta_s U n_U), n_U the double occupation of the proposed state on
 *   the orbitals with U != 0 (all of which must share one U), u = (z >> 11)
 *   2^-53, z = f(f(f(seed ^ step G) ^ parent) ^ h), f(x) the splitmix64 output
 *   function of x + G, G = 0x9E3779B97F4A7C15, step counted from 1.  Accepted
 *   states (each once, first occurrence in (parent rank, h) order) form the
 *   next frontier, whether new or not; new ones join F~ in that order until
 *   it holds n_f states.  An empty frontier is refilled with F~.  steps_out =
 *   steps taken; max_steps bounds them; burn_in is ignored.
 *   pre_level L > 0 (Sec. Subspace of the ground state, the speed-up by
 *   pre-accepting low double occupations; every orbital must be
 *   interacting): all sector states with n_U < L are accepted first -- they
 *   are enumerated level by level on the GPU (doubly occupied sites, then
 *   up-only, then down-only sites, each a ranked combination) -- and F~ and
 *   the first frontier are that set (start_key is then not used); if it
 *   already holds >= n_f states, F~ is its first n_f states in (n_U, key)
 *   order and steps_out = 0.  A level must hold < 2^31 states.
 * keys_dev: [cap] device output.  Returns MCD_E_CAPACITY if cap is too
 * small, MCD_E_SECTOR if start_key is not in the sector.  Scratch (visit
 * tables, sort buffers, frontier) comes from ws.  Synchronises.
 * ------------------------------------------------------------------------- */
typedef struct mcd_basis_cfg {
    int32_t mode;             /* MCD_BASIS_FULL or MCD_BASIS_CHAIN */
    int32_t n_up, n_dn;
    uint64_t start_key;       /* chain start state (in the sector) */
    uint64_t seed;
    double beta_s;            /* weight exp(-beta_s * E_diag) */
    int64_t burn_in;
    int64_t max_steps;        /* total steps, burn-in included */
    int64_t n_f;              /* target number of distinct states */
    int32_t pre_level;        /* MCD_BASIS_STEPS: pre-accept every state with
                                 n_U < pre_level (0 = none) */
} mcd_basis_cfg;

int mcd_basis_build(const mcd_model *model, const mcd_basis_cfg *cfg, uint64_t *keys_dev,
                    int64_t cap, int64_t *n_out, int64_t *steps_out, mcd_ws *ws, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_op_create -- the operator H~ = P H P on a basis (Eq.
 * h_matrix_projected; App. Lanczos, discarding out-of-basis states).
 *
 * keys_dev: [n] sorted unique keys of one or several (N_up, N_dn) sectors
 *   (a union of sectors is block diagonal).  Copied; the caller may free it.
 * storage: MCD_STORAGE_ON_THE_FLY recomputes every element at each apply
 *   (hop enumeration, popcount signs, hash lookup of the image state);
 *   MCD_STORAGE_CSR stores the matrix once as a packed CSR (one 32-bit word
 *   per nonzero: column, sign, amplitude class); MCD_STORAGE_AUTO picks CSR
 *   when it fits the format (n <= 2^(31 - ceil(log2 #classes)), <= 32 distinct
 *   |t|) and the workspace holds it, else on-the-fly.
 * validate != 0 checks on the GPU that the keys are sorted, unique and within
 *   n_orb bits (MCD_E_SECTOR otherwise).
 * ws: every buffer of the operator is taken from it and stays until
 *   mcd_op_destroy (which returns them).  A CSR operator also times its
 *   one-vector kernels and, when ws has room left, builds the grouped layout
 *   of kernels 7 / 8 (mcd_op_set_kernel).  Synchronises.
 * ------------------------------------------------------------------------- */
int mcd_op_create(const mcd_model *model, const uint64_t *keys_dev, int64_t n, int32_t storage,
                  int32_t validate, mcd_ws *ws, void *stream, mcd_op **out);
void mcd_op_destroy(mcd_op *op);

/* Workspace bytes mcd_op_create needs from an empty workspace, for keys_dev
 * [n] and `storage`.  On the fly: a closed form (ws may be NULL).  CSR (and
 * AUTO when the format fits): the count of kept hops is needed, so the index
 * is built and the nonzeros counted in the probe workspace ws; with ws NULL
 * or smaller than the probe the call returns MCD_E_WORKSPACE with *bytes =
 * the probe size.  *bytes covers the operator and its construction scratch;
 * *bytes_grouped (may be NULL) also the largest grouped layout, so that
 * mcd_op_create builds it.  Synchronises. */
int mcd_op_workspace_size(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                          int32_t storage, mcd_ws *ws, void *stream, size_t *bytes,
                          size_t *bytes_grouped);

typedef struct mcd_op_info_t {
    int64_t n;                /* basis size */
    int64_t nnz;              /* off-diagonal nonzeros (CSR), else -1 */
    int32_t storage;          /* resolved storage */
    int32_t n_classes;        /* distinct |t| amplitudes */
    int32_t rows_per_block;   /* CSR stream kernel row block */
    int32_t kernel;           /* one-vector CSR kernel (mcd_op_set_kernel numbering) */
    int64_t device_bytes;     /* device memory held by the operator */
    double build_ms;          /* time of index + CSR build */
    int64_t grouped_blocks;   /* row blocks of the grouped layout (kernels 7, 8); 0 = not
                                 built (on-the-fly operator, operator made for block
                                 products only, or a basis that does not fit the layout) */
    int64_t grouped_groups;   /* up-hop groups of the grouped layout (table entries) */
    int32_t rows_per_block_l; /* CSR: rows per block with <= 8192 nonzeros (tiles of the
                                 block products when the stream row block is shorter) */
    int32_t reserved;         /* 0 */
} mcd_op_info_t;

int mcd_op_info(const mcd_op *op, mcd_op_info_t *info);

/* Select the kernel of one-vector CSR products (y = H~ x with nvec = 1):
 *   1 = stream: one row block per workgroup, nonzeros staged through LDS;
 *   2 = merge-path: persistent workgroups over chunks of (nonzeros + rows),
 *       next chunk prefetched while the current one is reduced;
 *   3 = stream with an XCD-major workgroup order: each of the 8 XCDs walks
 *       one contiguous slice of rows, so its L2 serves mostly its own slice
 *       of x;
 *   4 = row-chunk: one thread per row, 16 column words then 16 gathers in
 *       flight per thread, no LDS staging (XCD-major row tiles);
 *   5 = stream with smaller row blocks (<= 1024 nonzeros per workgroup:
 *       less LDS and fewer loads per thread, for short rows);
 *   6 = 5 in XCD-major order;
 *   7 = grouped: the entries of each row block (<= 256 rows, <= 3072
 *       nonzeros) are stored in a second order in which up-spin hops are
 *       grouped by (source up string, target up string), so the lanes of a
 *       gather take the same hop of consecutive rows and read neighbouring
 *       x; each entry keeps its row-major slot, so every row still adds its
 *       terms in entry order (y bit-identical to kernel 1).  Built at
 *       creation when the basis has up-string segments of >= 16 rows on
 *       average, fewer than 2^28 rows, and every block fits 128 groups
 *       (mcd_op_info_t.grouped_blocks);
 *   8 = 7 in XCD-major order.
 * All give the same result up to summation order: kernels 1, 3, 5, 6, 7
 * and 8 add each row's terms in the same order (bit-identical y); 2 and 4
 * associate a row's sum differently (last-bit differences).  At creation a
 * CSR operator times every kernel on its own matrix and keeps the fastest,
 * so two operators of one basis may pick kernels of the two kinds: select
 * one here for results that are reproducible bit for bit across operators
 * and runs (a fixed kernel is deterministic).
 * MCD_E_INVALID for other values, an on-the-fly operator, or 7 / 8 on an
 * operator without the grouped layout. */
int mcd_op_set_kernel(mcd_op *op, int32_t kernel);

/* ---------------------------------------------------------------------------
 * mcd_hamiltonian_apply -- y = H~ x (the product every Lanczos step repeats,
 * Eq. next_vector; App. Lanczos).
 *
 * x_dev, y_dev: [n][nvec] row-major (vector k of row r at r*nvec + k), of
 *   type double (dtype MCD_F64) or float (MCD_F32, float accumulation).
 *   nvec in {1, 2, 4, 8, 16}.  x and y must not overlap.
 * Row r of y = d_r x_r + sum over kept hops, with d_r the diagonal energy.
 * Asynchronous on `stream`.
 * ------------------------------------------------------------------------- */
int mcd_hamiltonian_apply(const mcd_op *op, int32_t dtype, int32_t nvec, const void *x_dev,
                          void *y_dev, void *stream);

/* Diagonal <x_r|H|x_r> into diag_dev [n] (double).  Asynchronous. */
int mcd_hamiltonian_diagonal(const mcd_op *op, double *diag_dev, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_hamiltonian_connectivity -- the off-diagonal elements of rows
 * [row0, row1) as (row, col, value) triples, in the order the operator
 * enumerates them (up-spin hops in bond order, then down-spin hops in bond
 * order), for checking connectivity and signs exactly.  rows_dev, cols_dev:
 * int64 [cap]; vals_dev: double [cap].  count_out (host) = number of
 * triples; MCD_E_CAPACITY if cap is too small.  ws: 8 (row1 - row0) bytes of
 * scratch.  Synchronises.
 * ------------------------------------------------------------------------- */
int mcd_hamiltonian_connectivity(const mcd_op *op, int64_t row0, int64_t row1, int64_t *rows_dev,
                                 int64_t *cols_dev, double *vals_dev, int64_t cap,
                                 int64_t *count_out, mcd_ws *ws, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_hamiltonian_contract -- derivatives of H~ with respect to the model
 * parameters of Eq. hubbard_model, contracted with two vectors:
 *   d_t[q]   = <a| dH~/dt_q |b>   for every listed bond q (the hop operator of
 *              the pair, both spins and directions, restricted to the basis;
 *              bonds listed twice both receive the pair's value),
 *   d_U[i]   = <a| dH~/dU_i |b>   = sum_r a_r b_r n_{i up} n_{i dn},
 *   d_eps[i] = <a| dH~/deps_i |b> = sum_r a_r b_r (n_{i up} + n_{i dn}).
 * With a = b = the normalised ground state these are dE0/dtheta
 * (Hellmann-Feynman).  a_dev, b_dev: [n] double.  `model` must be the model
 * the operator was built from.  d_t [n_bonds], d_U [n_orb], d_eps [n_orb]:
 * host outputs (any may be NULL).  One pass on the GPU; workgroup partials
 * (8 (n_bonds + 2 n_orb) min(ceil(n / 256), 2048) bytes) come from ws.
 * Synchronises.
 * ------------------------------------------------------------------------- */
int mcd_hamiltonian_contract(const mcd_op *op, const mcd_model *model, const double *a_dev,
                             const double *b_dev, double *d_t, double *d_U, double *d_eps,
                             mcd_ws *ws, void *stream);

/* mcd_hamiltonian_contract for callers that cannot allocate or hand over
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid it): the same contraction and results, with its workgroup
 * partials in a fixed scratch array of the library in device memory (9.4 MB
 * per device, held until the process ends; up to MCD_MAX_BONDS + 2
 * MCD_MAX_ORB parameters, so every operator fits; MCD_E_CAPACITY otherwise).
 * Calls that overlap on one device race on that array: serialise them (one
 * stream, or wait for each call, which synchronises its stream).  Takes no
 * workspace and allocates nothing.  Synchronises. */
int mcd_hamiltonian_contract_noalloc(const mcd_op *op, const mcd_model *model,
                                     const double *a_dev, const double *b_dev, double *d_t,
                                     double *d_U, double *d_eps, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_lanczos_ground -- lowest eigenpair of H~ by Lanczos (App. Lanczos,
 * Eqs. next_vector / an_bn; ground state rebuilt by Eq. change_basis).
 *
 * Orthonormal recurrence v_{k+1} b_{k+1} = H v_k - a_k v_k - b_k v_{k-1} in
 * float64 with deterministic grid reductions; the tridiagonal H_eff is solved
 * on the host (Sturm bisection + inverse iteration) every check_every steps.
 * Stops when the Ritz residual b_{k+1} |s_k| <= tol max(1, |E0|), on
 * breakdown, or at max_iter (MCD_NOCONV, result still written).
 * phi0_dev: [n] start vector or NULL; NULL draws phi0[r] = 2u - 1 with u the
 *   top 53 bits of the first splitmix64 output of the state (seed XOR key_r).
 * psi0_dev: [n] output ground state (unit norm, float64), or NULL.  With
 *   store_vectors != 0 the Krylov vectors are kept in the workspace and psi0
 *   is one weighted sum; otherwise the recurrence is run a second time
 *   (Eq. change_basis without storage).
 * precision MCD_F64: float64 vectors throughout.  MCD_F32: the Krylov vectors
 *   and the product are float32 (float accumulation); the coefficients a_k,
 *   b_k, the tridiagonal solve and psi0's combination stay float64, and E0 is
 *   refined at the end by one float64 product: E0 = <psi0|H~|psi0> of the
 *   (float64, normalised) Ritz vector, with info->residual = ||H~ psi0 -
 *   E0 psi0|| from the same product.
 * alpha_out / beta_out: optional host arrays [max_iter] receiving a_k, b_{k+1}.
 * ws: scratch of mcd_lanczos_workspace_size bytes.  Returns MCD_E_NUMERIC if a
 * coefficient read back is not finite (a NaN / Inf in the input or the
 * operator).  Synchronises.
 * ------------------------------------------------------------------------- */
typedef struct mcd_lanczos_cfg {
    int32_t max_iter;
    int32_t check_every;      /* convergence test period (>= 1) */
    double tol;
    uint64_t seed;
    int32_t store_vectors;
    int32_t min_iter;         /* run at least this many steps */
    int32_t precision;        /* MCD_F64 or MCD_F32 (Krylov vectors) */
} mcd_lanczos_cfg;

typedef struct mcd_solve_info {
    int32_t iters;            /* Lanczos steps (or block steps) taken */
    int32_t converged;
    double e0;
    double residual;
    double solve_ms;          /* wall time of the call */
    double apply_ms;          /* time spent in H~ applies (events) */
    int32_t n_apply;
    int32_t krylov_dim;       /* band: number of Krylov vectors */
    int64_t n_plus, n_minus;  /* band: sizes of F~+ and F~- */
    int64_t n_truncated;      /* band: states kept by the w_t cut */
} mcd_solve_info;

int mcd_lanczos_ground(const mcd_op *op, const mcd_lanczos_cfg *cfg, const double *phi0_dev,
                       double *e0, double *psi0_dev, double *alpha_out, double *beta_out,
                       mcd_solve_info *info, mcd_ws *ws, void *stream);

/* Workspace bytes mcd_lanczos_ground needs with this operator and cfg. */
int mcd_lanczos_workspace_size(const mcd_op *op, const mcd_lanczos_cfg *cfg, size_t *bytes);

/* ---------------------------------------------------------------------------
 * mcd_batch_lanczos_ground -- ground states of n_ops independent operators at
 * once (App. Lanczos for each; e.g. bath-parameter instances of uneven basis
 * size).  Same recurrence, start vectors and stopping rule as
 * mcd_lanczos_ground, per operator; every step advances all unfinished
 * operators with a fixed set of launches (per-instance scalars, per-instance
 * deterministic reductions), and cfg->check_every steps are captured once
 * as a HIP graph and replayed.  The Krylov vectors of all operators are kept
 * (sum_i n_i (max_iter + 1) doubles; MCD_E_CAPACITY if they do not fit).
 * ops: [n_ops] CSR operators on the current device.  e0_out: host [n_ops].
 * psi0_dev: host array of n_ops device pointers ([n_i] doubles each) or NULL
 * (entries may be NULL).  iters_out: host [n_ops] or NULL.  ws: the Krylov
 * store and scratch (sum_i n_i (max_iter + 2) doubles and tables).  The graph
 * is captured on `stream`.  Synchronises.  MCD_NOCONV if any operator stopped
 * at max_iter.  cfg->precision must be MCD_F64.
 * ------------------------------------------------------------------------- */
int mcd_batch_lanczos_ground(mcd_op *const *ops, int32_t n_ops, const mcd_lanczos_cfg *cfg,
                             double *e0_out, double *const *psi0_dev, int32_t *iters_out,
                             mcd_solve_info *info, mcd_ws *ws, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_band_lanczos_green -- Green function of the truncated ground state on
 * Matsubara frequencies (Sec. Subspace of the Green function, Sec. Further
 * truncation, App. Band Lanczos).
 *
 * Steps: keep the most important states of psi0 up to weight w_t (order
 * |c|^2 descending, ties by key ascending; shortest prefix with cumulative
 * weight >= w_t; renormalise); build F~+ = union c+_mu F~ and F~- = union
 * c_mu F~ over the selected (orb[k], spin[k]) (Eq. excited_subspace); start
 * blocks c+_mu|psi0> and c_mu|psi0>; block Lanczos with block width
 * p = n_sel (the block Krylov space K_r^L of App. Band Lanczos),
 * reorthogonalisation against every stored block (cfg->reorth passes) and rank-revealing
 * deflation of directions with norm <= dtol max_k ||start_k||; then
 * G+_{mu nu}(i w) = [R^T (z - T)^-1 R]_{mu nu} at z = i w + E0 and
 * G-_{mu nu}(i w) = -[R^T (z - T)^-1 R] at z = E0 - i w (the resolvent form
 * of Eqs. green_qmatrix; R = start block in the Lanczos basis), evaluated by
 * a block continued fraction in complex128 on the host.  The particle and
 * hole runs advance in lockstep on `stream` (each block step's kernels are
 * enqueued for both runs before the next step).
 *
 * keys_dev [n], psi0_dev [n]: ground-state basis and vector (double).
 * orb, spin: [n_sel] host; spin 0 = up, 1 = down; n_sel <= 16.
 * omega: [n_freq] host frequencies: Matsubara w_n (cfg->eta <= 0, z = i w_n)
 *   or real w (cfg->eta > 0, z = w + i eta, the broadened real-frequency G
 *   of Sec. Green function whose -Im G_ii / pi is the density of states).
 * G_out, Gp_out, Gm_out: host complex128 interleaved [n_freq][n_sel][n_sel]
 *   (G = G+ + G-); Gp_out / Gm_out may be NULL.
 * precision MCD_F64: float64 Krylov blocks.  MCD_F32: float32 blocks and
 *   SpMM with float accumulation; Gram matrices, recurrence, deflation and
 *   the continued fraction stay float64.
 * max_blocks: block steps per run (Krylov dim <= max_blocks * p).
 * ws: every buffer of the call (cut, F~+- images, operators, Krylov blocks)
 *   is taken from it and returned before the call returns;
 *   mcd_band_workspace_size gives the bytes.  MCD_E_NUMERIC if psi0 has no
 *   finite nonzero weight or a recurrence coefficient read back is not
 *   finite.  Synchronises.
 * ------------------------------------------------------------------------- */
typedef struct mcd_band_cfg {
    int32_t max_blocks;
    int32_t precision;        /* MCD_F64 or MCD_F32 */
    double w_t;               /* target weight in (0, 1] */
    double dtol;              /* relative deflation tolerance (1e-10) */
    int32_t storage;          /* operator storage for F~+- */
    int32_t reorth;           /* passes of reorthogonalisation against every stored
                                 block: 2 (full, twice), 1 (once), 0 (none: only
                                 the three-term recurrence; 3 blocks kept) */
    int32_t per_column;       /* 1 = one single-vector product per block column
                                 (the unbatched reference form), 0 = block SpMM */
    double eta;               /* 0: Matsubara frequencies; > 0: real frequencies
                                 broadened by eta (the paper uses 0.05) */
    double g_tol;             /* > 0: stop a run once G at the check points (every
                                 frequency if <= 8, else the one nearest the real
                                 axis and 7 evenly spaced) changes by <= g_tol
                                 max|G| between checks 8 block steps apart;
                                 0: run max_blocks steps (or to exhaustion) */
    int32_t vjp_freq_batch;   /* derivative calls with regenerated blocks:
                                 frequencies per pass of the contraction (0: all
                                 in one pass); each pass holds two n x 2 batch p
                                 work matrices per sector */
    int32_t vjp_chunk;        /* derivative calls with regenerated blocks: Krylov
                                 blocks per accumulation
                                 (0: S2 / P blocks, at least 16, where S2 = 2
                                 batch p rounded up to 128 is the column count
                                 of a work matrix: a chunk then holds as many
                                 Krylov vectors as a work matrix has columns) */
} mcd_band_cfg;

int mcd_band_lanczos_green(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                           const double *psi0_dev, double e0, int32_t n_sel, const int32_t *orb,
                           const int32_t *spin, int32_t n_freq, const double *omega,
                           const mcd_band_cfg *cfg, double *G_out, double *Gp_out,
                           double *Gm_out, mcd_solve_info *info, mcd_ws *ws, void *stream);

/* Workspace bytes mcd_band_lanczos_green (keep = 0) or
 * mcd_band_lanczos_green_keep (keep != 0) needs from an empty workspace with
 * these arguments.  The sizes of F~+- and of their operators are data
 * dependent, so the call makes the cut, the images and both operators in the
 * probe workspace ws, replays the takes of the Krylov blocks on its host
 * bookkeeping, and releases everything (no block step is run).  If ws is too
 * small for that preparation it returns MCD_E_WORKSPACE with *bytes = a size
 * at which the failing request would have been served (grow ws and call
 * again).  Synchronises. */
int mcd_band_workspace_size(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                            const double *psi0_dev, double e0, int32_t n_sel, const int32_t *orb,
                            const int32_t *spin, int32_t n_freq, const double *omega,
                            const mcd_band_cfg *cfg, int32_t keep, mcd_ws *ws, void *stream,
                            size_t *bytes);

/* ---------------------------------------------------------------------------
 * mcd_band_lanczos_green_keep -- mcd_band_lanczos_green that also keeps the
 * two sector runs it makes (App. Band Lanczos: the Krylov blocks Q, the block
 * tridiagonal T, the operator on F~+-) for mcd_band_green_vjp_keep, so that
 * the derivative does not recompute them.
 *
 * Arguments and outputs as mcd_band_lanczos_green; cfg->w_t must be 1 and
 * cfg->per_column 0.  Every Krylov block is stored (max_blocks + 1 blocks of
 * n_x * P values per sector, P = n_sel rounded up to a power of two, in the
 * cfg->precision type), and all of it stays in ws until mcd_band_keep_destroy
 * (ws and its buffer must outlive the handle).  On success *keep_out is a new
 * handle owned by the caller; on error it is NULL and nothing is kept.
 * keys_dev and psi0_dev are not retained (the later derivative call passes
 * them again).  Synchronises.
 * ------------------------------------------------------------------------- */
typedef struct mcd_band_keep mcd_band_keep;
int mcd_band_lanczos_green_keep(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                                const double *psi0_dev, double e0, int32_t n_sel,
                                const int32_t *orb, const int32_t *spin, int32_t n_freq,
                                const double *omega, const mcd_band_cfg *cfg, double *G_out,
                                double *Gp_out, double *Gm_out, mcd_solve_info *info,
                                mcd_ws *ws, void *stream, mcd_band_keep **keep_out);

/* Releases a handle of mcd_band_lanczos_green_keep (NULL is ignored): its
 * pieces go back to the workspace of the forward call.  No call on the handle
 * may be running. */
void mcd_band_keep_destroy(mcd_band_keep *keep);

/* ---------------------------------------------------------------------------
 * mcd_batch_band_green -- mcd_band_lanczos_green for many independent
 * instances (bath-parameter sets of a quantum impurity model, each with its
 * own basis and ground state), same selection, frequencies and cfg.
 *
 * All runs (particle and hole of every instance) advance in lockstep: each
 * kernel of a block step is enqueued for every unfinished run before the
 * next, on `stream`, with one synchronisation every 8 block steps for the
 * ranks and convergence checks of all of them.  Instances are prepared (cut,
 * F~+-, operators) and run in groups of as many as ws holds at once.  Each
 * instance's result is computed exactly as by mcd_band_lanczos_green
 * (bit-identical: a run's arithmetic does not depend on the other runs).
 *
 * models, keys_dev, n, psi0_dev, e0: [n_inst] per-instance inputs (device
 *   keys / psi0 as in mcd_band_lanczos_green); G_out: [n_inst] host
 *   complex128 outputs [n_freq][n_sel][n_sel] (G = G+ + G-).
 * info (optional): iters = max over instances, krylov_dim / n_plus / n_minus /
 *   n_truncated summed, solve_ms = wall time of the batch.
 * ws: must hold at least the largest single instance (MCD_E_WORKSPACE
 *   otherwise).  Synchronises.
 * ------------------------------------------------------------------------- */
int mcd_batch_band_green(const mcd_model *const *models, const uint64_t *const *keys_dev,
                         const int64_t *n, const double *const *psi0_dev, const double *e0,
                         int32_t n_inst, int32_t n_sel, const int32_t *orb, const int32_t *spin,
                         int32_t n_freq, const double *omega, const mcd_band_cfg *cfg,
                         double *const *G_out, mcd_solve_info *info, mcd_ws *ws, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_band_green_vjp -- reverse-mode derivative of the Green function (and of
 * E0) with respect to the Hamiltonian's parameters theta = (t_b, U_i, eps_i)
 * of Eq. hubbard_model, for the G that mcd_band_lanczos_green returns with
 * the same arguments.
 *
 * For a real function L(G, E0) with G_bar[f][mu][nu] = dL/dRe G + i dL/dIm G
 * (the gradient convention of torch for complex tensors) and e0_bar =
 * dL/dE0, writes dL/dtheta = Re sum conj(G_bar) dG/dtheta + e0_bar dE0/dtheta.
 * G+(z) = B^T (z - H+)^-1 B with B = c+|psi0>, z = E0 + zeta (G- likewise
 * with minus signs), so dG/dtheta has three parts, all evaluated here:
 *   * the resolvent:  X^T (dH/dtheta - dE0/dtheta) X, X = (z - H)^-1 B,
 *     through the Krylov blocks Q (X = Q S, S from the block tridiagonal
 *     T): tr(Q^T dH/dtheta Q M) - tr(M) dE0/dtheta with M = Re sum_f S_f
 *     conj(G_bar_f)^T S_f^T = sg A B^T (A, B: m P x 2 n_freq p real).  With
 *     every block stored: Z = Q (M + M^T) (one MFMA product) and the trace
 *     as the symmetric contraction of Q with Z, each hop pair once.  With
 *     the blocks regenerated: tr(U^T dH/dtheta V), U = Q (sg A), V = Q B
 *     accumulated over chunks of blocks (MFMA products) and contracted per
 *     batch of frequencies.  The two forms agree to rounding;
 *   * dE0/dtheta = <psi0| dH/dtheta |psi0> (Hellmann-Feynman);
 *   * the response of the start block through d psi0/dtheta =
 *     -(H - E0)^+ dH/dtheta psi0: one conjugate-gradient solve
 *     (H - E0) xi = P lambda on F~ (P projects out psi0, lambda collects the
 *     adjoint of the start blocks), then -<xi| dH/dtheta |psi0>.
 * The Krylov blocks are recomputed here (mcd_band_green_vjp_keep instead
 * takes them from a forward call that kept them): with cfg->reorth > 0 the
 * recomputed runs store every block (max_blocks + 1 blocks of n_x * P
 * values per sector, as reorthogonalisation needs them anyway); with
 * cfg->reorth = 0 no block is stored: a second pass of the same recurrence
 * regenerates Q_0, Q_1, ... one at a time (three ring blocks and a chunk of
 * cfg->vjp_chunk blocks in memory), with the same numbers bit for bit.
 *
 * psi0_dev: the normalised, non-degenerate ground state; cfg->w_t must be 1
 *   (a target-weight cut is not differentiable).
 * G_bar: host complex128 [n_freq][n_sel][n_sel].
 * d_t [n_bonds] (listed bonds; a pair listed twice gets the pair's
 *   derivative in both entries), d_U [n_orb], d_eps [n_orb]: host outputs.
 * info: iters = conjugate-gradient iterations, residual = its relative
 *   residual, krylov_dim, n_plus, n_minus, solve_ms.
 * cg_tol: relative residual of the solve (1e-12 is typical); cg_max_iter.
 * ws: the scratch of the call (ground-sector operator, solve vectors; with
 *   a store Z, n_x x m P values rounded up to 128 columns; with regenerated
 *   blocks the work matrices U and V, n_x x 2 batch p values each, rounded
 *   up to 128 columns, batch = cfg->vjp_freq_batch or n_freq, and a chunk of
 *   blocks; without a kept forward also the two sector runs).
 * Returns MCD_NOCONV (outputs filled) if the solve stopped at cg_max_iter,
 * MCD_E_BREAKDOWN if it met <p, (H - E0) p> <= 0 (psi0 is not a
 * non-degenerate ground state of H~: the response is undefined).
 * Synchronises.
 * ------------------------------------------------------------------------- */
int mcd_band_green_vjp(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                       const double *psi0_dev, double e0, int32_t n_sel, const int32_t *orb,
                       const int32_t *spin, int32_t n_freq, const double *omega,
                       const mcd_band_cfg *cfg, const double *G_bar, double e0_bar,
                       double cg_tol, int32_t cg_max_iter, double *d_t, double *d_U,
                       double *d_eps, mcd_solve_info *info, mcd_ws *ws, void *stream);

/* ---------------------------------------------------------------------------
 * mcd_band_green_vjp_keep -- mcd_band_green_vjp on the sector runs kept by
 * mcd_band_lanczos_green_keep instead of recomputed ones.  The arguments are
 * those of mcd_band_green_vjp and must equal the kept forward call's (n,
 * e0, selection, frequencies, and cfg's max_blocks, precision, dtol,
 * storage, reorth, eta, g_tol; else MCD_E_INVALID); keys_dev, psi0_dev and
 * model must be the same data.  The results are those of mcd_band_green_vjp
 * (the kept runs are the runs it would recompute).  keep is not consumed and
 * may serve several calls, one at a time (they share its scratch blocks).
 * ws: this call's scratch (the kept runs stay in the forward call's
 * workspace).  Synchronises.
 * ------------------------------------------------------------------------- */
int mcd_band_green_vjp_keep(const mcd_model *model, const uint64_t *keys_dev, int64_t n,
                            const double *psi0_dev, double e0, int32_t n_sel, const int32_t *orb,
                            const int32_t *spin, int32_t n_freq, const double *omega,
                            const mcd_band_cfg *cfg, const double *G_bar, double e0_bar,
                            double cg_tol, int32_t cg_max_iter, double *d_t, double *d_U,
                            double *d_eps, mcd_solve_info *info, mcd_ws *ws, void *stream,
                            mcd_band_keep *keep);

#ifdef __cplusplus
}
#endif
#endif /* MCD_H */
