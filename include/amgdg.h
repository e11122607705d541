/*
 * amgdg -- geometric adaptive smoothed-aggregation multigrid for DG matrices
 * (Pan, Lindsey & Persson, "Geometric adaptive smoothed aggregation multigrid
 * for discontinuous Galerkin discretisations", arXiv 2504.13373), on one AMD
 * Instinct MI355X (gfx950).
 *
 * The problem (Section 4.5): given the n x n DG matrix A with one dense nb x nb
 * block per element and coupled element pair, the mesh graph of the elements
 * and a nested hierarchy of element aggregates (Section 4.1), build the
 * multigrid operators of Algorithm 5 and solve A x = b with the V-cycle of
 * Algorithm 2, on its own or as a preconditioner of a Krylov method.
 *
 * Conventions for every entry point
 *  - Return value: AMGDG_OK (0) on success, a negative AMGDG_E* code on error,
 *    AMGDG_ENOCONV (> 0) when a solve stopped at its iteration limit.  No entry
 *    point throws; amgdg_last_error() gives a message for the calling thread.
 *  - Host arrays are read during the call only (the library copies what it
 *    keeps).  Device arrays are caller-owned and must stay valid until the work
 *    queued on `stream` has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *    device work is queued on it; calls that return host data synchronise it.
 *  - Block storage is row-major inside each block; multi-column vectors are
 *    row-major n x m (the m values of one dof are contiguous).
 *  - Element and dof numbering is the caller's.  The library renumbers elements
 *    internally so that every aggregate is a contiguous range; this is invisible
 *    except through the AMGDG_INTERNAL_ORDER flag of amgdg_apply.
 *  - A handle is not thread-safe; distinct handles are.
 */
#ifndef AMGDG_H
#define AMGDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define AMGDG_OK            0
#define AMGDG_EINVAL       -1  /* bad argument: null pointer, size, unsorted or duplicate
                                  column, missing diagonal block, non-nested hierarchy */
#define AMGDG_ESINGULAR    -2  /* a diagonal block or the coarsest matrix has a pivot
                                  |u_ii| <= n * eps * max|a| */
#define AMGDG_ENOMEM       -3  /* device or host allocation failed */
#define AMGDG_EHIP         -4  /* HIP runtime error */
#define AMGDG_ENAN         -5  /* NaN or Inf in the data or the iteration */
#define AMGDG_EBREAKDOWN   -6  /* Krylov breakdown, e.g. p^T A p <= 0 in CG */
#define AMGDG_EUNSUPPORTED -7  /* valid input outside what the library implements */
#define AMGDG_ENOCONV       1  /* iteration limit reached; x holds the last iterate */

/* --------------------------------------------------------------- parameters */
typedef struct {
    int32_t  n_levels;     /* levels L_0..L_{n_levels-1}; L_{n_levels-1} is solved directly */
    int32_t  r;            /* adaptive candidates per level (columns of B^k), 1..64 */
    int32_t  t_pre;        /* pre-smoothing sweeps (Algorithm 2) */
    int32_t  t_post;       /* post-smoothing sweeps */
    int32_t  q_power;      /* power-iteration steps of Algorithm 4 */
    int32_t  relax_max;    /* cap on the sweeps of the candidate relaxation (eq:bsmooth) */
    double   omega_fixed;  /* > 0: use this damping on every level instead of eq:omega */
    double   gamma;        /* stagnation tolerance of eq:bsmooth */
    double   n_cut;        /* coarsening factor of eq:sik (h-step) */
    int32_t  b_update;     /* 0: B^{k+1} = R B^k (Algorithm 5); 1: P~^T B^k (eq:SA_Bk) */
    int32_t  mixed;        /* 1: also keep FP32 copies of all level operators */
    uint64_t pow_seed;     /* level k's power-iteration start vector: SplitMix64 stream
                              pow_seed + k, entries 2u-1, in caller dof order */
    uint64_t b1_seed;      /* B^1 stream when no B^1 is given (Box-Muller normals) */
    double   delta;        /* h*-step threshold of eq:sik: an aggregate that equals its only
                              child keeps the singular vectors above delta * sigma_1 */
    int32_t  hstar_smooth; /* a replicated level (every aggregate one unit: the h*-step of
                              Algorithm 5): 0 takes T = P~ (its coarse operator keeps the fine
                              stencil, as the paper's printed h*-hierarchy implies), 1 smooths
                              P~ as in eq:TR0 */
    int32_t  matfree_levels; /* kappa of Section 4.6: levels 1..kappa (at most n_levels-2) keep
                              no A_k after the setup; the V-cycle applies A_k as
                              R_{k-1} A_{k-1} T_{k-1} (eq:matfree1, eq:matfree2), down to A_0.
                              Single steps that need A_k are then EUNSUPPORTED on those levels */
    int32_t  restrict_resid; /* 1 (default): on levels whose coarse block size is at most 4 and
                              where it holds no more values than the residual pass over
                              D_k^{-1} A_k and R_k D_k it replaces (plus 2^21), keep
                              M_k = R_k (D_k - omega_k A_k); the V-cycle's last pre-sweep then
                              also writes the residual it starts from, e, and the coarse right-hand
                              side is M_k e = R_k (b_k - A_k u) (Algorithm 2, reassociated: one
                              product over D_k^{-1} A_k fewer per level and cycle).  0: residual,
                              then R_k D_k.  Needs t_pre >= 1; not on matrix-free levels */
} amgdg_params;

/* Fills the paper's defaults: gamma 0.03 (Section 4.2), q 3 (Section 4.4),
 * t_pre = t_post = 3 (Section 5), n_cut 3 (2D value 2^d - d + 1, Section 4.3),
 * delta 1e-3 (Section 4.3), relax_max 100, r 3, n_levels 2, adaptive omega,
 * B^{k+1} = R B^k, FP64 only. */
void amgdg_default_params(amgdg_params* p);

/* ------------------------------------------------------------ hierarchy */
/* Nested element aggregates by recursive coordinate bisection, the stand-in for
 * the 2^d-way METIS splits of Section 4.1.  A node splits along the axis of
 * largest centroid extent (ties: lowest axis), elements sorted by (coordinate,
 * element id), left child = first ceil(m/2).  With D = ceil(log2 n_elem), the
 * level-k aggregates (k >= 1) are the nodes at depth D - k*bisections (a leaf
 * above that depth is its own aggregate), numbered depth first.
 *   centroids : host, n_elem x dim doubles (dim 1..3)
 *   agg_out   : host, (n_levels-1) x n_elem int32: row k-1 maps element -> level-k aggregate
 *   leaf_order: host, n_elem int64 or NULL: elements in depth-first leaf order
 * Host only; never touches the GPU.  EINVAL if D - (n_levels-1)*bisections < 0. */
int amgdg_partition_rcb(int64_t n_elem, int32_t dim, const double* centroids, int32_t n_levels,
                        int32_t bisections, int32_t* agg_out, int64_t* leaf_order);

/* ------------------------------------------------- symbolic plan (host only) */
/* The index construction of the setup, without numbers: element renumbering,
 * and per level the block patterns of T (eq:TR0: block (e,J) iff J is the
 * aggregate of e or of a block column of row e of A_k), R = T^T and
 * A_{k+1} = R A_k T (block (I,J) iff T(a,I), A_k(a,b), T(b,J) all exist).
 * On a replicated level (every aggregate a single unit) T = P~: row e of T holds
 * its own aggregate only (amgdg_params.hstar_smooth = 0, the default).
 * Inputs as for amgdg_setup.  Host only; never touches the GPU. */
typedef struct amgdg_plan_s* amgdg_plan;
int amgdg_plan_create(amgdg_plan* out, int64_t n_elem, const int32_t* row_ptr, const int32_t* col_idx,
                      int64_t nnzb, int32_t n_levels, const int32_t* agg_of_elem);
void amgdg_plan_destroy(amgdg_plan p);

/* Items for amgdg_plan_size / amgdg_plan_export and amgdg_export_level.  Level-0
 * rows (A_0, T_0, D_0^{-1}, B^0, P~_0) are returned in caller element order;
 * coarse levels are numbered by aggregate id. */
#define AMGDG_PERM        1   /* int64[n_elem]: internal position -> caller element (level 0 only) */
#define AMGDG_T_ROWPTR    2   /* int32[n_units_k + 1] */
#define AMGDG_T_COLIDX    3   /* int32[nnzb_T] (level-(k+1) aggregate ids) */
#define AMGDG_A_ROWPTR    4   /* int32[n_units_k + 1]: pattern of A_k (k = 0: the caller's) */
#define AMGDG_A_COLIDX    5
#define AMGDG_R_ROWPTR    6   /* int32[n_agg + 1] */
#define AMGDG_R_COLIDX    7
#define AMGDG_A_VALS     10   /* double[nnzb_A * nb * nb] (A_k) */
#define AMGDG_T_VALS     11   /* double[nnzb_T * nb * s] */
#define AMGDG_R_VALS     12   /* double[nnzb_T * s * nb] */
#define AMGDG_DINV       13   /* double[n_units * nb * nb] */
#define AMGDG_B_RELAXED  14   /* double[n * r]: candidates after relaxation */
#define AMGDG_B_INPUT    15   /* double[n * r]: candidates before relaxation */
#define AMGDG_PTILDE     16   /* double[n_units * nb * s]: the P~ rows of each unit */
#define AMGDG_SVALS      17   /* double[n_agg * r]: singular values, descending (zeros beyond
                                 the rank bound min(|A_J|, r)) */
#define AMGDG_UNIT_DOFS  18   /* int32[n_units]: dofs of each unit of level k (s_J on coarse levels;
                                 a unit's vector rows beyond them are zero padding) */
#define AMGDG_M_ROWPTR   19   /* int32[n_agg + 1]: pattern of M_k = R_k (D_k - omega_k A_k), that of
                                 R_k A_k (block (I,c) iff R_k(I,e) and A_k(e,c) for some e) */
#define AMGDG_M_COLIDX   20   /* int32[nnzb_M] (level-k units) */
#define AMGDG_M_VALS     21   /* double[nnzb_M * s * nb]; level export only */
/* The plan exports the M pattern of every level; a handle exports the three M
 * items only on levels that keep M_k (amgdg_level_info.restrict_resid = 1), and
 * returns EUNSUPPORTED elsewhere. */

/* Number of elements of `what` (in its own type) at level k. */
int amgdg_plan_size(amgdg_plan p, int32_t k, int32_t what, int64_t* count);
int amgdg_plan_export(amgdg_plan p, int32_t k, int32_t what, void* host_buf, int64_t bytes);

/* ------------------------------------------------------------------ setup */
typedef struct amgdg_ctx* amgdg_handle;

/* Algorithm 5 on the GPU: per level k = 0..n_levels-2 the block-Jacobi diagonal
 * inverses (Section 4.4), the damping (Algorithm 4, eq:omega), the relaxation of
 * the candidates (eq:bsmooth), the tentative prolongator by per-aggregate SVD
 * (eq:splitB_dg, eq:sik), T = (I - omega D^{-1} A) P~ and R = T^T (eq:TR0),
 * A_{k+1} = R A_k T and B^{k+1} = R B^k; then the inverse of the coarsest
 * matrix.  Every arithmetic step runs in the library's HIP kernels.
 *   n_elem, nb       : element count and dofs per element (1..64)
 *   row_ptr, col_idx : host BSR pattern, int32, columns sorted, diagonal present
 *   vals             : host, nnzb * nb * nb doubles
 *   adj_ptr, adj_idx : host face graph of the elements (CSR) or NULL; only checked
 *   agg_of_elem      : host, (n_levels-1) x n_elem, element -> level-k aggregate;
 *                      ids dense per level, nested, and ordered so that the
 *                      children of each coarser aggregate have consecutive ids
 *   B1               : host, n x r row-major in caller order, or NULL
 *   p                : parameters (NULL: defaults)
 * Coarse sizes (eq:sik) are chosen per aggregate J: s_J = min(ceil(|A_J| / n_cut),
 * |A_J|, r) when J has several children (h-step), and the number of singular
 * values above delta times the largest when J equals its only child (h*-step:
 * pass a level whose aggregates are the previous level's units, numbered so
 * that the next level's children stay consecutive).  A coarse level whose
 * units differ in size stores every unit with the level's largest s_J; the
 * rows beyond a unit's own s_J are zero in every operator and vector (a unit
 * diagonal keeps D invertible there), and AMGDG_UNIT_DOFS reports the sizes.
 * r must be 1..64, an aggregate may hold at most 1024 dofs and s_J at most 64
 * (EUNSUPPORTED otherwise). */
int amgdg_setup(amgdg_handle* out, int64_t n_elem, int32_t nb, const int32_t* row_ptr,
                const int32_t* col_idx, const double* vals, int64_t nnzb, const int32_t* adj_ptr,
                const int32_t* adj_idx, const int32_t* agg_of_elem, const amgdg_params* p,
                const double* B1, void* stream);
int amgdg_destroy(amgdg_handle h);

typedef struct {
    int64_t n_units;     /* block rows of A_k */
    int32_t nb;          /* block size of level k (the largest unit) */
    int32_t s;           /* block size of level k+1: the largest s_J (0 on the coarsest level) */
    int64_t n;           /* dofs of level k */
    int64_t nnzb;        /* blocks of A_k */
    int64_t nnzb_T;      /* blocks of T_k (0 on the coarsest level) */
    int64_t n_agg;       /* block rows of A_{k+1} */
    double  omega;       /* damping omega_k */
    double  rho;         /* power-iteration estimate (NaN if omega was fixed) */
    int32_t r;           /* candidates relaxed on this level */
    int32_t sweeps[64];  /* relaxation sweeps per candidate */
    int64_t bytes_A, bytes_Dinv, bytes_T, bytes_R;   /* FP64 bytes held for level k */
    int64_t n_dofs;      /* dofs of level k without the padding of units below nb (= n when
                            every unit holds nb) */
    int32_t matfree;     /* 1: A_k is applied matrix-free (not stored) */
    int64_t bytes_handle;/* device bytes held by the whole hierarchy (every level) */
    int64_t nnzb_M;      /* blocks of M_k = R_k (D_k - omega_k A_k) where it is kept, else 0 */
    int32_t restrict_resid; /* 1: the V-cycle restricts through M_k (amgdg_params.restrict_resid) */
    int64_t bytes_M;     /* FP64 bytes of M_k (0 when not kept) */
    int64_t nnzb_S;      /* blocks stored for D_k^{-1} A_k: its off-diagonal ones (its diagonal
                            blocks are the identity and are applied as such; 0 on a
                            matrix-free level) */
} amgdg_level_info;
int amgdg_level_info_get(amgdg_handle h, int32_t k, amgdg_level_info* out);
int amgdg_num_levels(amgdg_handle h);

/* Copies an item of level k to host memory (synchronises `stream`). */
int amgdg_export_level(amgdg_handle h, int32_t k, int32_t what, void* host_buf, int64_t bytes,
                       void* stream);

/* ------------------------------------------------------------------ solve */
#define AMGDG_FP64  0   /* FP64 V-cycle */
#define AMGDG_MIXED 1   /* FP32 V-cycle (FP32 operators and accumulation; coarsest
                           solve in FP64) inside FP64 outer iterations */

#define AMGDG_STATIONARY 0  /* x <- x + V(b - A x) (Algorithm 2 as a solver) */
#define AMGDG_PCG        1  /* preconditioned CG (symmetric positive definite A) */
#define AMGDG_FCG        2  /* flexible CG (Polak-Ribiere beta) */
#define AMGDG_FGMRES     3  /* restarted right-preconditioned FGMRES(restart), CGS2;
                               each restart recomputes the FP64 residual */

typedef struct {
    int32_t iterations[64];   /* per column (first 64) */
    double  rel_residual[64]; /* true ||b - A x|| / ||b|| per column, FP64 */
    int32_t max_iterations;
    int32_t all_converged;
    double  seconds;
} amgdg_solve_stats;

/* Solves A X = B for m columns from X = 0 (or the given X if AMGDG_X0 is set in
 * flags), stopping each column when its true relative residual is <= rtol.
 *   b_dev, x_dev : device, n x m doubles (row-major: column c of row i at
 *                  i * m + c), caller order
 *   stats        : host or NULL
 * The V-cycle precision is AMGDG_FP64 or AMGDG_MIXED (needs params.mixed).
 * PCG and FCG (section 5 runs CG with the V-cycle of Algorithm 2 as its
 * preconditioner) treat the columns as independent solves: every kernel
 * computes column c from column c alone and reductions add in an order fixed
 * by n, so a column's iterates, iteration count and result are bit-identical
 * whatever m is and whatever the other columns hold.  In FCG a column whose
 * recursive residual has dropped by 1e-6 since its last check, or meets rtol,
 * is checked against its true residual, which replaces the recursive one when
 * it is above rtol.  Returns AMGDG_ENOCONV if a column did not converge within
 * max_it iterations; a breakdown (p^T A p <= 0) or a NaN fails the call. */
#define AMGDG_X0             1
#define AMGDG_INTERNAL_ORDER 2
#define AMGDG_EAGER          4  /* launch the V-cycle kernel by kernel instead of replaying
                                   its captured HIP graph.  Without it, solve and vcycle replay
                                   the graph unless one pass over the level-0 operator
                                   S_0 = D^{-1} A_0 reads 128 MB or more (in the V-cycle's
                                   precision): there the host queues the kernels well ahead
                                   of the device, and the graph's start and end would only
                                   add idle time.  The results are the same either way. */
int amgdg_solve(amgdg_handle h, int32_t m, const double* b_dev, double* x_dev, int32_t method,
                int32_t precision, double rtol, int32_t max_it, int32_t restart, int32_t flags,
                amgdg_solve_stats* stats, void* stream);

/* One V-cycle z = V(r) from z = 0 (Algorithm 2, one pass), m columns.
 * precision AMGDG_FP64: r, z are double*; AMGDG_MIXED: float*.
 * On level k the first pre-smoothing sweep (from u = 0) forms omega D^{-1} b_k
 * and keeps c = D^{-1} b_k; every later sweep is u + omega (c - S_k u) with
 * S_k = D^{-1} A_k precomputed at setup, and the restricted residual is
 * (R_k D)(c - S_k u), the same operator as Algorithm 1's sweep and
 * R_k (b_k - A_k u) with one matrix read per sweep instead of A_k and D^{-1};
 * on a level that keeps M_k = R_k (D_k - omega_k A_k) (params.restrict_resid)
 * it is M_k e with e = c - S_k u the residual the last pre-sweep starts from,
 * which that sweep writes.  Consecutive passes over S_k run in opposite
 * directions (the order rows are visited in; the arithmetic of a row does not
 * depend on it).  Into a non-coarsest coarse level the restriction also
 * applies that level's D^{-1} (its first sweep's operations), so b_{k+1} is
 * not stored. */
int amgdg_vcycle(amgdg_handle h, int32_t m, const void* r_dev, void* z_dev, int32_t precision,
                 int32_t flags, void* stream);

/* The V-cycle of amgdg_vcycle, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It allocates nothing: its level vectors (and, for caller-order
 * vectors, the two permuted copies of level 0) live in one static workspace
 * of 128 MiB per GPU, part of the library's code object and held by each GPU
 * the library runs on until the process ends.  The kernels are those of
 * amgdg_vcycle, launched one by one on `stream` (no graph), so z is
 * bit-identical to amgdg_vcycle's.  Arguments as for amgdg_vcycle
 * (AMGDG_EAGER is implied).  AMGDG_EUNSUPPORTED, before any work is queued, if
 * the vectors need more than the workspace holds (about
 * (4 n_0 + 5 sum_{0<k<N} n_k + 2 n_N + 2 n_0) m words).  Every call on a GPU
 * shares that GPU's workspace: calls whose work overlaps on one GPU (other
 * streams, other host threads) race and must be ordered by the caller. */
int amgdg_vcycle_static(amgdg_handle h, int32_t m, const void* r_dev, void* z_dev, int32_t precision,
                        int32_t flags, void* stream);

/* Single steps of the hot path on level k (one kernel launch each, for tests
 * and timing).  x, b, y: device arrays of the sizes below, double (FP64) or
 * float (MIXED), m columns.  An argument the operation does not read (b for
 * SPMV, RESTRICT, COARSE; x for SWEEP0) is ignored and may be NULL.  Level-0
 * vectors are in caller order unless AMGDG_INTERNAL_ORDER is set (then no
 * permutation kernel runs).  y must not alias x or b. */
#define AMGDG_OP_SPMV      0  /* y = A_k x                               (n_k)      */
#define AMGDG_OP_SWEEP     1  /* y = x + omega D^{-1} (b - A_k x)         (Alg. 1)   */
#define AMGDG_OP_SWEEP0    2  /* y = omega D^{-1} b (sweep from zero)                */
#define AMGDG_OP_RESIDUAL  3  /* y = b - A_k x                                       */
#define AMGDG_OP_RESTRICT  4  /* y = R_k x   (x: n_k, y: n_{k+1})                    */
#define AMGDG_OP_PROLONG   5  /* y = b + T_k x (x: n_{k+1}, b, y: n_k)               */
#define AMGDG_OP_COARSE    6  /* y = A_N^{-1} x on the coarsest level (always FP64)  */
/* The forms the V-cycle runs (its sweeps after the first, and its restriction,
 * on the row-scaled operators; b here is the scaled right-hand side D^{-1} b_k): */
#define AMGDG_OP_SWEEP_SCALED    7  /* y = x + omega (b - D^{-1} A_k x)               */
#define AMGDG_OP_RESTRICT_SCALED 8  /* y = R_k D x  (x: n_k, y: n_{k+1})              */
/* The forms of the restricted residual (amgdg_params.restrict_resid): */
#define AMGDG_OP_RESTRICT_RESID  9  /* y = R_k (D - omega A_k) x (x: n_k, y: n_{k+1});
                                       EUNSUPPORTED on a level that keeps no M_k  */
#define AMGDG_OP_SWEEP_SCALED_RESID 10 /* y[0 : n_k m] = x + omega (b - D^{-1} A_k x) and
                                       y[n_k m : 2 n_k m] = b - D^{-1} A_k x: y holds
                                       2 n_k m values                            */
int amgdg_apply(amgdg_handle h, int32_t k, int32_t op, int32_t m, int32_t precision, const void* x,
                const void* b, void* y, int32_t flags, void* stream);

/* Device bytes of the solve state of one batch of `width` right-hand sides on
 * this hierarchy, with an FGMRES basis of `restart` vectors if restart > 0
 * (what a server counts against its budget per batch: CG batches have the
 * server's width and restart 0, FGMRES batches width 1). */
int amgdg_batch_bytes(amgdg_handle h, int32_t width, int32_t restart, int64_t* bytes);

/* Serving: continuous batching of the PCG / FCG / FGMRES solves of
 * amgdg_solve (section 5), submitted one right-hand side at a time.
 * CG requests on the same (handle, method, precision) share a batch of `width`
 * columns: a request takes a free column between two iterations and leaves it
 * when it converges, fails or reaches max_it, so every level operator is read
 * once per iteration for all requests of the batch (the multi-RHS kernels).
 * An FGMRES request takes a batch of one column with its Krylov basis.
 * Each request's iterates, iteration count and x are bit-identical to
 * amgdg_solve of that right-hand side alone (m = 1).  Each batch runs on a
 * stream of its own, so the work of different batches overlaps.  A new batch is created only while the device bytes of
 * all batches (amgdg_batch_bytes) stay within hbm_budget_bytes; an idle batch
 * of another key is released to make room; otherwise the request waits.
 * Requests are admitted in submission order; one that cannot be placed does
 * not hold back those that can.  The server does not own the handles: destroy
 * it before them.  One host thread drives a server.
 *   width           : columns per batch, 1..64
 *   hbm_budget_bytes: > 0 */
typedef struct amgdg_server_s* amgdg_server;
int amgdg_server_create(amgdg_server* out, int32_t width, int64_t hbm_budget_bytes);
/* Queues one right-hand side.  b_dev, x_dev: device, n doubles each, caller
 * order unless AMGDG_INTERNAL_ORDER; with AMGDG_X0, x_dev holds the initial
 * guess.  b_dev must hold its values on the device when submitted (the
 * server's streams are not ordered after the caller's) and both arrays must
 * stay valid and untouched until the request is reported by amgdg_server_poll,
 * when x_dev holds the result.  tag: the caller's id, reported back.  method: AMGDG_PCG, AMGDG_FCG or AMGDG_FGMRES
 * (restart 1..256, ignored otherwise).  AMGDG_ENOMEM if one batch on this
 * handle exceeds the budget. */
int amgdg_server_submit(amgdg_server s, amgdg_handle h, const double* b_dev, double* x_dev,
                        int32_t method, int32_t precision, double rtol, int32_t max_it, int32_t restart,
                        int32_t flags, int64_t tag);
/* Admits queued requests and advances every batch whose last queued
 * iteration has finished, without blocking; with wait != 0 it first waits
 * (spinning) until at least one batch has moved on.  n_pending (may be NULL):
 * requests queued, running or not yet reported. */
int amgdg_server_step(amgdg_server s, int32_t wait, int64_t* n_pending);
/* Reports up to `capacity` finished requests, oldest first, and forgets them:
 * tag, status (AMGDG_OK, AMGDG_ENOCONV, AMGDG_EBREAKDOWN, AMGDG_ENAN), iteration
 * count, true relative residual and latency (seconds from submission to the
 * step that saw x written).  Arrays are host memory of `capacity` entries;
 * all but tags may be NULL.  *n_done: entries written. */
int amgdg_server_poll(amgdg_server s, int32_t capacity, int64_t* tags, int32_t* status,
                      int32_t* iterations, double* rel_residual, double* latency_s, int32_t* n_done);
/* Waits for the server's streams and frees its batches. */
int amgdg_server_destroy(amgdg_server s);

/* Autotuner: picks the launch shapes for m columns (1..64) by timing the
 * candidates on the operators of this hierarchy's V-cycle (HIP events on
 * `stream`):
 *   - columns per launch of the sliced and block-CSR kernels (1, 2, 4, 8, 16);
 *   - operand blocks loaded ahead in the 16-column MFMA tiles (1, 2, 4; 3 as well where the tiles
 *     stage their operands in LDS, whose chunk of blocks this sizes);
 *   - with AMGDG_TUNE_LANES, the lanes per block row of every block-CSR
 *     operator (4..64, 128, 256; timed at one column).
 * The first two never change a result.  The lane-group width changes the
 * summation order, hence rounding, of the block-CSR products: it can be tuned
 * once per handle (AMGDG_EINVAL on a second attempt), before use, and then
 * holds for every column count, so columns stay independent of m.  Drops the
 * handle's captured V-cycles; not to be called while a server uses the
 * handle.  Untuned shapes: 4 (FP64) / 8 (FP32) columns per sliced launch, 16
 * per block-CSR launch, 4 MFMA blocks ahead, and lanes per block row the power
 * of two >= the mean blocks per row (4..64), or, for rows of 96 or more
 * entries, lanes over the row's entries: a wavefront per block row (128), or a
 * workgroup of four (256) for rows of 128 or more entries on operators of
 * fewer than 4,096 block rows. */
#define AMGDG_TUNE_LANES 1
int amgdg_autotune(amgdg_handle h, int32_t m, int32_t flags, void* stream);
/* The shapes in use on level k (0..levels-2) for m columns, out[16]:
 * [0..3) lanes per block row of A_k, T_k, R_k (0: sliced layout; 128 and 256:
 * a wavefront or a workgroup per block row, lanes over its entries); D^{-1} A_k
 * and R_k D, the operators the V-cycle runs, share the shapes of A_k and R_k;
 * [3..6) FP64 and [6..9) FP32 columns per launch (0: default rule);
 * [9..12) FP64 and [12..15) FP32 MFMA blocks loaded ahead (0: default 4);
 * [15] 1 if the lane widths were tuned. */
int amgdg_tuning_get(amgdg_handle h, int32_t k, int32_t m, int32_t* out);

/* Message for the last non-zero status returned on the calling thread. */
const char* amgdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AMGDG_H */
