// Launch wrappers of the HIP kernels (gfx950, wave64).  All launches go to the
// stream given; nothing here allocates or synchronises.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgdg {

// Sliced, row-interleaved block-sparse matrix with br x bc blocks (br > 4).
//
// Block rows are grouped in slices of G rows (floor(64 / br), fewer for long
// rows: see sell_rows_per_wave); one wavefront owns a slice and each of its first L = G * br lanes owns one scalar row.  A
// slice stores K (its longest block row) block slots per row, padded with zero
// blocks whose column is 0.  The K*bc values of a lane's row are flattened as
// t = k*bc + j and stored in vectors of VW = 16 / sizeof(T) values:
//     vals[voff[s] + (t / VW) * L * VW + l * VW + t % VW]
// so that one 16-byte load per lane reads VW values and a wavefront reads one
// contiguous run of 16 * L bytes.  The column of slot k of block row g of the
// slice is cols[coff[s] + k * G + g].  tpad is the largest K*bc of any slice
// rounded up to VW (the per-row length of the x staging buffer in LDS).
// Block row g of slice s is block row s * G + g, or rows[s * G + g] when rows
// is set (rows sorted by length within windows of slices, so that a slice's
// rows have similar lengths; n_brow marks an empty position).
template <typename T>
struct Sell {
    int32_t n_brow = 0, br = 0, bc = 0, G = 0, L = 0, n_slices = 0, tpad = 0, brpad = 0;
    const int64_t* voff = nullptr;
    const int32_t* coff = nullptr;
    const int32_t* K = nullptr;
    const int32_t* cols = nullptr;
    const T* vals = nullptr;
    const int32_t* rows = nullptr;
    int32_t unit = 0;  // see below
    // per launch (k_spmv): 1 visits each XCD's run of slices from its end, so
    // that a pass that follows one in the other direction first reads what the
    // memory-side cache took in last; the result does not depend on it
    int32_t rev = 0;
};
// unit (Sell, Bcsr, Nbsr): 1 for a square operator whose diagonal blocks are
// the identity and are not stored, S = D^{-1} A: every product adds the row's
// own x entries to the stored blocks' sum

// Block-CSR matrix with small br x bc blocks (br <= 4), for coarse levels and
// restriction: a group of P lanes (P a power of two, 4..64) owns one block row,
// lane p of the group handles blocks rp[row] + p, + P, ...; the partial
// products are summed across the group with xor-shuffles.
template <typename T>
struct Bcsr {
    // P: 4..64 lanes per block row, each lane taking whole blocks; 128 one
    // wavefront per block row and 256 one workgroup (four wavefronts) per block
    // row, whose lanes take the row's entries (block, column) in order: for rows
    // of many blocks, so that neighbouring lanes read neighbouring values
    int32_t n_brow = 0, br = 0, bc = 0, P = 0;
    const int32_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const T* vals = nullptr;  // row-major blocks
    int32_t unit = 0;
};
constexpr int BCSR_MAXBR = 4;

// Block-sparse matrix in its natural layout (row-major br x bc blocks, block
// CSR rp/ci), read by the MFMA product of 16-column tiles (br, bc <= 16).
template <typename T>
struct Nbsr {
    int32_t n_brow = 0, br = 0, bc = 0;
    const int32_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const T* vals = nullptr;
    int32_t unit = 0;
};
constexpr int MFMA_COLS = 16;
constexpr int NBSR_MAXB = 16;

// sweep modes
enum SweepMode : int {
    SWEEP = 0,   // y = x + omega D^{-1} (b - A x)
    SWEEP0 = 1,  // y = omega D^{-1} b; with y2, also y2 = D^{-1} b
    RELAX = 2,   // y = x - omega D^{-1} A x   (columns with mask 0 are copied)
    DINVA = 3,   // y = D^{-1} A x
};
// spmv modes
enum SpmvMode : int {
    AX = 0,      // y = A x
    B_MINUS = 1, // y = b - A x
    B_PLUS = 2,  // y = b + A x
    S_SWEEP = 3, // y = x + omega (b - A x): the block-Jacobi sweep on the row-scaled
                 // operator A = D^{-1} A_k, with b = D^{-1} b_k
    AX_DOT = 4,  // y = A x, and one partial of x . y per workgroup and column (launch_spmv_dot)
    AX_DSCALE = 5, // y = omega D'^{-1} (A x), y2 = D'^{-1} (A x), D'^{-1} the br x br blocks of the
                   // output rows (block CSR only): a restriction that starts the coarse smoothing
    S_SWEEP_R = 6, // S_SWEEP that also writes y2 = b - A x, the residual of the iterate it starts from
};

// D^{-1} in sliced layout: the br x br block of block row g is stored like a
// one-slot slice with its columns padded to brpad (a multiple of VW):
// value (i, j) at dinv[s * brpad * L + (j / VW) * L * VW + (g * br + i) * VW + j % VW].
// `cap` bounds the columns processed per launch (1, 2, 4, 8; 0: 4 FP64 / 8 FP32);
// it does not change the arithmetic of any column.
// y2 (SWEEP0 only, may be null) receives D^{-1} b.  omega is read by S_SWEEP only.
template <typename T>
hipError_t launch_sweep(int mode, const Sell<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega,
                        int m, const int32_t* colmask, hipStream_t st, int cap = 0, T* y2 = nullptr);
template <typename T>
hipError_t launch_spmv(int mode, const Sell<T>& A, const T* x, const T* b, T* y, int m, hipStream_t st, int cap = 0,
                       T omega = T(0), T* y2 = nullptr);  // y2: S_SWEEP_R only (required there)
// Block rows per wavefront of the sliced layout: floor(64 / br), lowered until
// one column of FP64 x staging plus D^{-1} (rows of up to max_row_blocks blocks
// of bc columns) fits the 64 KB of LDS a workgroup may take; at least 1, and 1
// when lowering leaves half the lanes or more idle (br <= 16: the split-row
// kernels then keep all 64 lanes busy).  A
// launch whose staging exceeds the device's per-workgroup LDS even at one
// block row per wavefront stages x in chunks of 512 values (one column per
// launch).
int sell_rows_per_wave(int br, int bc, int max_row_blocks);
// y = A x and xy[c] = x[:,c] . y[:,c] (FP64, sliced layout): each workgroup of
// the product writes one partial sum per column (its four slices in order) to
// part (n_slices * 8 doubles suffice), which a one-workgroup kernel adds in a
// fixed order (the same for every column count)
hipError_t launch_spmv_dot(const Sell<double>& A, const double* x, double* y, int m, double* part, double* xy,
                           hipStream_t st, int cap = 0);
// the same operations on a block-CSR matrix; dinv: natural layout (n_brow x br x br);
// cap: 1, 2, 4, 8 or 16 columns per launch (0: 16)
template <typename T>
hipError_t launch_bsweep(int mode, const Bcsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega, int m,
                         const int32_t* colmask, hipStream_t st, int cap = 0, T* y2 = nullptr);
template <typename T>
hipError_t launch_bspmv(int mode, const Bcsr<T>& A, const T* x, const T* b, T* y, int m, hipStream_t st,
                        int cap = 0, T omega = T(0), const T* dinv = nullptr, T* y2 = nullptr);

// MFMA products of 16-column tiles (m a multiple of 16, row-major n x m
// vectors): one wavefront per block row computes the block row's br x 16 tile
// of A x with 16x16x4 matrix instructions (FP32 or FP64 accumulation, the
// type of T); then, by mode:
//   MF_AX y = A x, MF_BMINUS y = b - A x, MF_BPLUS y = b + A x,
//   MF_SWEEP y = x + omega D^{-1} (b - A x), MF_SWEEP0 y = omega D^{-1} b (and
//   y2 = D^{-1} b when y2 is not null), MF_SSWEEP y = x + omega (b - A x),
//   MF_RDINV y = omega D^{-1} (A x), y2 = D^{-1} (A x),
//   MF_SSWEEP_R y = x + omega (b - A x) and y2 = b - A x
// with D^{-1} natural (n_brow x br x br, row-major), applied by MFMA too.
enum MfmaMode : int {
    MF_AX = 0, MF_BMINUS = 1, MF_BPLUS = 2, MF_SWEEP = 3, MF_SWEEP0 = 4, MF_SSWEEP = 5, MF_RDINV = 6, MF_SSWEEP_R = 7,
    MF_AXDOT = 8  // y = A x and per-workgroup partials of x . y (launch_mfma_dot only)
};
// u: blocks whose operand fragments are loaded before their products (1, 2 or 4;
// 0: 4); for the tiles that stage their operands in LDS, the register budget of
// a chunk of blocks (16 x 16 u values of operand and of x rows; u = 3 for them
// only, a chunk of four 10 x 10 blocks); it does not change the arithmetic.
template <typename T>
hipError_t launch_mfma(int mode, const Nbsr<T>& A, const T* dinv, const T* x, const T* b, T* y, T omega, int m,
                       hipStream_t st, int u = 0, T* y2 = nullptr);
// y = A x and xy[c] = x[:,c] . y[:,c] on the FP64 tiles (m a multiple of 16),
// one launch per 16-column tile: each workgroup writes one partial per column
// (its four block rows in order, each block row's rows in order), a second
// kernel adds every KRY_BLOCKS-th of them in a fixed order, and k_finalize
// adds those.  part: mfma_dot_parts(A.n_brow) doubles, part2: 16 * KRY_BLOCKS.
int64_t mfma_dot_parts(int64_t n_brow);
hipError_t launch_mfma_dot(const Nbsr<double>& A, const double* x, double* y, int m, double* part, double* part2,
                           double* xy, hipStream_t st, int u = 0);

// Block-Jacobi steps on a level applied matrix-free (q = A_k u from a chain of
// products), D^{-1} natural (n_units x nb x nb), m columns row-major:
//   BD_SWEEP y = x + omega (c - D^{-1} q), BD_RESID y = c - D^{-1} q,
//   BD_START y = omega D^{-1} q and y2 = D^{-1} q (q = b, from zero).
enum BdiagMode : int { BD_SWEEP = 0, BD_RESID = 1, BD_START = 2 };
template <typename T>
hipError_t launch_bdiag(int mode, const T* dinv, const T* q, const T* c, const T* x, T* y, T* y2, T omega,
                        int64_t n_units, int nb, int m, hipStream_t st);

// ---- setup ----
// Fill the sliced values of type T from natural FP64 blocks: for slot q (one
// block slot of one block row), its source block src[q] (-1: zero padding),
// its slice's value offset base[q], its slot k[q] and row-in-slice g[q].
template <typename T>
hipError_t launch_to_sell_vals(const double* nat, const int64_t* slot_src, const int64_t* slot_base,
                               const int32_t* slot_k, const int32_t* slot_g, int64_t n_slots, int L, int br, int bc,
                               T* vals, hipStream_t st);
// pos[e] (may be null: e) is the slice position s * G + g of block row e
template <typename T>
hipError_t launch_dinv_to_sell(const double* dinv_nat, int64_t n_brow, int br, int G, int L, int brpad, T* dinv_sell,
                               hipStream_t st, const int32_t* pos = nullptr);
hipError_t launch_f64_to_f32(const double* a, float* b, int64_t n, hipStream_t st);
// nb 1..64 (nb > 16: one wavefront per block, the block in LDS)
hipError_t launch_block_inverse(const double* Avals, const int32_t* diag_pos, int64_t n_brow, int nb, double* dinv,
                                int32_t* flag, hipStream_t st);
hipError_t launch_svd(const double* B, int r, const int32_t* first_child, int64_t n_agg, int nb, int s,
                      double* Pu, double* svals, int32_t* flag, hipStream_t st);
// Per-aggregate SVD for up to 64 candidates and any aggregate size (one
// workgroup per aggregate, working columns in `work` at offsets woff[J]:
// nr * r doubles, plus nr * nr when nr < r).  Unit u of the level owns the
// rows u * nb + [0, sz[u]).  sJ[J] >= 0: vectors kept; sJ[J] < 0: keep those
// with singular value above delta times the largest (written back to sJ).
// Pu (row-major, spad columns) must be zeroed before.  flag |= 2 for more
// than 1024 rows or a count above spad, 4 for a zero singular value kept.
hipError_t launch_svd_gen(const double* B, int r, const int32_t* first_child, const int32_t* sz, int nb,
                          int64_t n_agg, int32_t* sJ, double delta, int spad, double* work, const int64_t* woff,
                          double* Pu, double* svals, int32_t* flag, hipStream_t st);
// unit diagonal on the padding rows i >= sz[u] of every diagonal block
hipError_t launch_pad_diag(double* Avals, const int32_t* diag_pos, int64_t n_brow, int nb, const int32_t* sz,
                           hipStream_t st);
hipError_t launch_T_build(const double* Avals, const int32_t* A_ci, const int32_t* T_row, const int32_t* T_ci,
                          const int32_t* Tm_ptr, const int32_t* Tm_a, const int32_t* agg, int64_t nT, int nb, int s,
                          const double* Pu, const double* dinv, double omega, double* W, double* Tvals,
                          hipStream_t st);
hipError_t launch_R_from_T(const double* Tvals, const int32_t* R_t, int64_t nR, int nb, int s, double* Rvals,
                           hipStream_t st);
// out block b = vals block src[b] (n blocks of `per` values)
hipError_t launch_gather_blocks(const double* vals, const int32_t* src, int64_t n, int per, double* out,
                                hipStream_t st);
// S = D^{-1} A block row by block row (S has A's pattern; dinv natural)
hipError_t launch_row_scale(const double* Avals, const int32_t* rp, int64_t n_brow, int nb, const double* dinv,
                            double* Svals, hipStream_t st);
// RD = R D with D the diagonal blocks of A (A_diag: position of block row i's
// diagonal block in Avals); RD has R's pattern
hipError_t launch_right_diag(const double* Rvals, const int32_t* R_ci, int64_t nR, int nb, int s, const double* Avals,
                             const int32_t* A_diag, double* RDvals, hipStream_t st);
hipError_t launch_AT(const double* Avals, const double* Tvals, const int64_t* pp, const int32_t* pa,
                     const int32_t* pt, int64_t nAT, int nb, int s, double* ATvals, hipStream_t st);
hipError_t launch_galerkin(const double* Tvals, const double* ATvals, const int64_t* pp, const int32_t* pt,
                           const int32_t* pu, int64_t nC, int nb, int s, double* Cvals, hipStream_t st);
// M = R (D - omega A), block v (s x nb) = sum over pairs q in [pp[v], pp[v+1]) of
// w_q R_{pr[q]} A_{pa[q]}, w_q = 1 - omega when the A block is diagonal (the R
// block's column R_ci[pr[q]] equals M_ci[v]), else -omega
hipError_t launch_restrict_resid(const double* Rvals, const double* Avals, const int32_t* R_ci, const int32_t* M_ci,
                                 const int64_t* pp, const int32_t* pr, const int32_t* pa, int64_t nM, int nb, int s,
                                 double omega, double* Mvals, hipStream_t st);
hipError_t launch_dense_from_bsr(const double* vals, const int32_t* rp, const int32_t* ci, int64_t n_brow, int nb,
                                 int64_t nnzb, double* dense, hipStream_t st);
// in-place inverse of a dense row-major n x n matrix (Gauss-Jordan, row pivoting);
// flag |= 1 if a pivot is <= tol_scale * amax[0]; rowc, colc: n doubles of scratch
hipError_t launch_gj_invert(double* a, int64_t n, int32_t* piv, int32_t* flag, const double* amax, double tol_scale,
                            double* rowc, double* colc, hipStream_t st);
// out[0] = max |a_i|; out must hold 1 + DOT_PARTS doubles
hipError_t launch_absmax(const double* a, int64_t n, double* out, hipStream_t st);
hipError_t launch_uniform(uint64_t seed, const int64_t* perm, int64_t n_units, int nb, double* x, hipStream_t st);
// a level whose units have sz[u] <= nb real dofs, the first at real offset roff[u]
hipError_t launch_uniform_padded(uint64_t seed, const int64_t* roff, const int32_t* sz, int64_t n_units, int nb,
                                 double* x, hipStream_t st);
hipError_t launch_normal(uint64_t seed, const int64_t* perm, int64_t n_units, int nb, int r, double* x,
                         hipStream_t st);

constexpr int DOT_PARTS = 1024;
// ---- vectors ----
// per-column dot products of row-major n x m arrays, accumulated in FP64 in a
// fixed order: out[c] = sum_i a[i,c] * b[i,c]
template <typename T>
hipError_t launch_dot(const T* a, const T* b, int64_t n, int m, double* part, double* out, hipStream_t st);
// y[i,c] = a*x[i,c] + by*y[i,c] with per-column device scalars (alpha[c] * sa)
hipError_t launch_axpby_dev(const double* x, double* y, int64_t n, int m, const double* alpha, double sa,
                            double by, hipStream_t st);
// ---- fused Krylov steps (deterministic: each workgroup writes partial sums,
// a one-workgroup finalize kernel adds them in a fixed order) ----
constexpr int KRY_BLOCKS = 2048;
// out[c] = sum_i a[i,c] b[i,c]   (part: 2 * 16 * KRY_BLOCKS doubles)
hipError_t launch_dot_tail(const double* a, const double* b, int64_t n, int m, double* part, double* out,
                           hipStream_t st);
// CG update of m columns: alpha = active ? rz / pq : 0 (flag[c] |= 1 if an active pq <= 0,
// 2 if alpha or rr[c] is not finite); x += alpha p; r_out = r_in - alpha q; r32 = float(r_out)
// if r32 != NULL; rr[c] = ||r_out[:,c]||^2.  flag holds one int32 per column.
// With stat_host (pinned host memory), the last finalize also copies the
// stat_len doubles at stat (device) there, after rr and the flags are final.
hipError_t launch_cg_update(double* x, const double* r_in, double* r_out, const double* p, const double* q,
                            float* r32, int64_t n, int m, const double* rz, const double* pq,
                            const int32_t* active, double* part, double* rr, int32_t* flag, hipStream_t st,
                            const double* stat = nullptr, double* stat_host = nullptr, int stat_len = 0);
// z = double(z32) if z32 != NULL (z is then only written, and may be NULL);
// rz[c] = r.z ; zro[c] = z.r_old if r_old != NULL
hipError_t launch_zdots(const float* z32, double* z, const double* r, const double* r_old, int64_t n, int m,
                        double* part, double* rz, double* zro, hipStream_t st);
// p = z + beta p, beta = active ? (rz_new - zro) / rz_old : 0  (zro may be NULL);
// with z32 != NULL, z is double(z32) and the z argument is not read
hipError_t launch_cg_dir(double* p, const double* z, int64_t n, int m, const double* rz_new, const double* zro,
                         const double* rz_old, const int32_t* active, hipStream_t st, const float* z32 = nullptr);

// Column c of a batch (row-major n x ld arrays kb, kx, r, p, q) takes a new
// right-hand side: kb = r = b (caller column, stride ldb, rows reordered by perm
// if perm != NULL), kx = x0 (same addressing, or 0 if x0 == NULL), p = q = 0,
// flag[c] = 0.
hipError_t launch_admit(const double* b, int64_t ldb, const double* x0, int64_t ldx, const int64_t* perm,
                        int64_t n_units, int nb, double* kb, double* kx, double* r, double* p, double* q, int ld,
                        int c, int32_t* flag, hipStream_t st);
// out[row(i) * ldo] = in[i * ldi], row(i) = perm[i / nb] * nb + i % nb (i if perm == NULL)
hipError_t launch_scatter_col(const double* in, int64_t ldi, double* out, int64_t ldo, const int64_t* perm,
                              int64_t n_units, int nb, hipStream_t st);
// dst[i,c] = src[i,c] for the columns c with mask[c] != 0
hipError_t launch_copy_cols(const double* src, double* dst, int64_t n, int m, const int32_t* mask, hipStream_t st);
// y = Ainv x (dense, row-major n x n, FP64, FP64 sums), m columns; V = float
// vectors are widened on load and the result is rounded once on store
template <typename V>
hipError_t launch_gemv(const double* Ainv, const V* x, V* y, int64_t n, int m, hipStream_t st);
// level-0 reorder: out[internal unit u] = in[caller element perm[u]] (gather) or the inverse (scatter)
template <typename Ti, typename To>
hipError_t launch_permute(const Ti* in, To* out, const int64_t* perm, int64_t n_units, int nb, int m,
                          int gather, hipStream_t st);
template <typename Ti, typename To>
hipError_t launch_convert(const Ti* in, To* out, int64_t n, hipStream_t st);
hipError_t launch_scale_by_inv_norm(double* x, int64_t n, const double* nrm2, hipStream_t st);
// Krylov multi-vector ops (FGMRES): h[j] = V[j] . w for j < nv (V: nv x n); w -= sum_j V[j] h[j]
hipError_t launch_multidot(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* part,
                           double* out, hipStream_t st);
hipError_t launch_multi_axpy(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t n,
                             double sign, hipStream_t st);

}  // namespace amgdg
