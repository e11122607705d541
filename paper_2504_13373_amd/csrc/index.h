// Host-side index construction of the multigrid setup: hierarchy checks,
// element renumbering and the symbolic (pattern-only) phase of eq:TR0 and of
// the Galerkin product.  No HIP here: this part runs and is tested on the CPU.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace amgdg {

// Patterns of one level transition k -> k+1, all in internal numbering (level-k
// units renumbered so that every aggregate is a contiguous range of units).
struct LevelPattern {
    int64_t n_units = 0;   // units (block rows) of level k
    int64_t n_agg = 0;     // units of level k+1
    std::vector<int32_t> agg;          // unit -> aggregate
    std::vector<int32_t> first_child;  // aggregate J owns units [first_child[J], first_child[J+1])

    // A_k
    std::vector<int32_t> A_rp, A_ci;
    std::vector<int32_t> A_diag;       // block index of the diagonal block of each row

    bool replicated = false;           // every aggregate is a single unit (h*-step)
    // T_k = P~ - omega D^{-1} (A_k P~): block (e, J)
    std::vector<int32_t> T_rp, T_ci;
    std::vector<int32_t> T_row;        // block row of each T block
    std::vector<int32_t> Tm_ptr, Tm_a; // A blocks (e, c) with agg(c) == J, per T block

    // R_k = T_k^T: block (J, e), and the T block it transposes
    std::vector<int32_t> R_rp, R_ci, R_t;

    // AT = A_k T_k: block (e, J) = sum over pairs (a, t) of A_a * T_t
    std::vector<int32_t> AT_rp, AT_ci;
    std::vector<int64_t> AT_pp;
    std::vector<int32_t> AT_pa, AT_pt;

    // A_{k+1} = R_k (A_k T_k): block (I, J) = sum over pairs (t, u) of T_t^T * AT_u
    std::vector<int32_t> C_rp, C_ci;
    std::vector<int64_t> C_pp;
    std::vector<int32_t> C_pt, C_pu;

    // M_k = R_k (D_k - omega A_k): block (I, c) = sum over pairs (r, a) of
    // R_r * A_a, r = (I, e) a block of R and a = (e, c) a block of A_k; A_k's
    // diagonal blocks enter with weight 1 - omega, the others with -omega.
    // It restricts the residual after a block-Jacobi sweep from the residual
    // before it: R D (c - S u') = M (c - S u) for u' = u + omega (c - S u).
    // Formed on demand (symbolic_M): only levels that keep M, and exports, need it.
    bool M_done = false;
    std::vector<int32_t> M_rp, M_ci;
    std::vector<int64_t> M_pp;
    std::vector<int32_t> M_pr, M_pa;
};

struct Plan {
    int64_t n_elem = 0;
    int32_t n_levels = 0;
    std::vector<int64_t> perm;    // internal unit -> caller element (level 0)
    std::vector<int64_t> iperm;   // caller element -> internal unit
    std::vector<int64_t> A0_src;  // internal level-0 block -> caller block index
    std::vector<LevelPattern> lv; // n_levels - 1 transitions
    // pattern of the coarsest operator
    std::vector<int32_t> AN_rp, AN_ci, AN_diag;
};

// Throws std::invalid_argument with a message on invalid input.  A level whose
// aggregates are its own units (a replicated level, the h*-step) takes T = P~
// (T row e holds its own aggregate only) unless hstar_smooth is set, which
// applies eq:TR0's smoothing pattern there too.
void build_plan(Plan& P, int64_t n_elem, const int32_t* row_ptr, const int32_t* col_idx, int64_t nnzb,
                int32_t n_levels, const int32_t* agg_of_elem, bool hstar_smooth = false);

// The pattern of M_k = R_k (D_k - omega A_k) and its pairs (once per level).
void symbolic_M(LevelPattern& L);

void rcb_partition(int64_t n_elem, int32_t dim, const double* cent, int32_t n_levels, int32_t bisections,
                   int32_t* agg_out, int64_t* leaf_out);

}  // namespace amgdg
