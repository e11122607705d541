// Host-side index construction: recursive coordinate bisection, hierarchy
// validation, element renumbering and the symbolic phase of the setup.
//
// Patterns follow eq:TR0 and the Galerkin product A_{k+1} = R A_k T (Section
// 4.2) structurally: no numerical dropping, so a block exists iff some product
// of existing blocks lands on it.
#include "index.h"

#include <algorithm>
#include <array>
#include <numeric>
#include <stdexcept>

namespace amgdg {

static void fail(const std::string& m) { throw std::invalid_argument(m); }

// ----------------------------------------------------------------------- RCB

void rcb_partition(int64_t n, int32_t dim, const double* cent, int32_t n_levels, int32_t b,
                   int32_t* agg_out, int64_t* leaf_out) {
    if (n < 1 || dim < 1 || dim > 3 || n_levels < 1 || b < 1 || !cent) fail("rcb: bad arguments");
    int D = 0;
    while ((int64_t(1) << D) < n) ++D;
    if (n_levels > 1 && D - (n_levels - 1) * b < 0) fail("rcb: too many levels for this mesh");
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<int64_t> start = {0, n}, next;
    for (int depth = 0; depth <= D; ++depth) {
        for (int k = 1; k < n_levels; ++k) {
            if (depth != D - k * b || !agg_out) continue;
            int32_t* out = agg_out + int64_t(k - 1) * n;
            for (size_t s = 0; s + 1 < start.size(); ++s)
                for (int64_t i = start[s]; i < start[s + 1]; ++i) out[perm[i]] = int32_t(s);
        }
        if (depth == D) break;
        next.clear();
        for (size_t s = 0; s + 1 < start.size(); ++s) {
            int64_t s0 = start[s], s1 = start[s + 1], m = s1 - s0;
            next.push_back(s0);
            if (m < 2) continue;
            double lo[3], hi[3];
            for (int a = 0; a < dim; ++a) lo[a] = hi[a] = cent[perm[s0] * dim + a];
            for (int64_t i = s0 + 1; i < s1; ++i)
                for (int a = 0; a < dim; ++a) {
                    double v = cent[perm[i] * dim + a];
                    lo[a] = std::min(lo[a], v);
                    hi[a] = std::max(hi[a], v);
                }
            int axis = 0;
            double best = hi[0] - lo[0];
            for (int a = 1; a < dim; ++a)
                if (hi[a] - lo[a] > best) { best = hi[a] - lo[a]; axis = a; }
            std::sort(perm.begin() + s0, perm.begin() + s1, [&](int64_t x, int64_t y) {
                double cx = cent[x * dim + axis], cy = cent[y * dim + axis];
                return cx < cy || (cx == cy && x < y);
            });
            next.push_back(s0 + (m + 1) / 2);
        }
        next.push_back(n);
        start.swap(next);
    }
    if (leaf_out) std::copy(perm.begin(), perm.end(), leaf_out);
}

// ------------------------------------------------------------- symbolic phase

// T pattern: row e holds {agg(e)} U {agg(c) : c in cols(A[e,:])}; with the A
// blocks that feed each T block.  own_only: row e holds {agg(e)} alone (T = P~).
static void symbolic_T(LevelPattern& L, bool own_only) {
    const int64_t nu = L.n_units;
    L.T_rp.assign(nu + 1, 0);
    std::vector<std::pair<int32_t, int32_t>> ent;  // (J, a) ; a = -1 for the own aggregate
    std::vector<int32_t> ci, mptr, ma, trow;
    std::vector<int32_t> mcount;
    for (int64_t e = 0; e < nu; ++e) {
        ent.clear();
        ent.push_back({L.agg[e], -1});
        if (!own_only)
            for (int32_t a = L.A_rp[e]; a < L.A_rp[e + 1]; ++a) ent.push_back({L.agg[L.A_ci[a]], a});
        std::stable_sort(ent.begin(), ent.end(),
                         [](const auto& x, const auto& y) { return x.first < y.first || (x.first == y.first && x.second < y.second); });
        for (size_t i = 0; i < ent.size();) {
            size_t j = i;
            ci.push_back(ent[i].first);
            trow.push_back(int32_t(e));
            int32_t cnt = 0;
            for (; j < ent.size() && ent[j].first == ent[i].first; ++j)
                if (ent[j].second >= 0) { ma.push_back(ent[j].second); ++cnt; }
            mcount.push_back(cnt);
            i = j;
        }
        L.T_rp[e + 1] = int32_t(ci.size());
    }
    L.T_ci.swap(ci);
    L.T_row.swap(trow);
    L.Tm_ptr.assign(L.T_ci.size() + 1, 0);
    for (size_t t = 0; t < mcount.size(); ++t) L.Tm_ptr[t + 1] = L.Tm_ptr[t] + mcount[t];
    L.Tm_a.swap(ma);
}

// R = T^T pattern with the source T block of every R block (rows = aggregates,
// columns = units in increasing order).
static void symbolic_R(LevelPattern& L) {
    const int64_t nt = int64_t(L.T_ci.size());
    L.R_rp.assign(L.n_agg + 1, 0);
    for (int64_t t = 0; t < nt; ++t) L.R_rp[L.T_ci[t] + 1]++;
    for (int64_t J = 0; J < L.n_agg; ++J) L.R_rp[J + 1] += L.R_rp[J];
    L.R_ci.resize(nt);
    L.R_t.resize(nt);
    std::vector<int32_t> fill(L.R_rp.begin(), L.R_rp.end() - 1);
    for (int64_t e = 0; e < L.n_units; ++e)
        for (int32_t t = L.T_rp[e]; t < L.T_rp[e + 1]; ++t) {
            int32_t p = fill[L.T_ci[t]]++;
            L.R_ci[p] = int32_t(e);
            L.R_t[p] = t;
        }
}

// Rows of a product pattern with their pairs: for each output row, visit(emit)
// calls emit(col, p1, p2) for every contributing pair in a fixed order; the
// row's distinct columns are sorted and each column's pairs keep the visit
// order (the order a sort of (col, p1, p2) triples gives when the visit runs
// p1, then p2, ascending and meets each (p1, col) once).
template <typename Visit>
static void product_rows(int64_t n_rows, int64_t n_cols, std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                         std::vector<int64_t>& pp, std::vector<int32_t>& p1, std::vector<int32_t>& p2,
                         Visit visit) {
    rp.assign(size_t(n_rows) + 1, 0);
    pp.assign(1, 0);
    ci.clear();
    p1.clear();
    p2.clear();
    std::vector<int64_t> mark(size_t(n_cols), -1), start(size_t(n_cols), 0);
    std::vector<int32_t> cnt(size_t(n_cols), 0), cols;
    for (int64_t I = 0; I < n_rows; ++I) {
        cols.clear();
        visit(I, [&](int32_t c, int32_t, int32_t) {
            if (mark[c] != I) {
                mark[c] = I;
                cnt[c] = 0;
                cols.push_back(c);
            }
            ++cnt[c];
        });
        std::sort(cols.begin(), cols.end());
        int64_t pos = int64_t(p1.size());
        for (int32_t c : cols) {
            start[c] = pos;
            pos += cnt[c];
            ci.push_back(c);
            pp.push_back(pos);
        }
        p1.resize(size_t(pos));
        p2.resize(size_t(pos));
        visit(I, [&](int32_t c, int32_t a, int32_t b) {
            const int64_t q = start[c]++;
            p1[size_t(q)] = a;
            p2[size_t(q)] = b;
        });
        if (ci.size() >= (size_t(1) << 31)) fail("plan: a product pattern exceeds int32 indexing");
        rp[size_t(I) + 1] = int32_t(ci.size());
    }
}

// AT = A T: row e, block J = sum over (a = (e,c), t = (c,J)).
static void symbolic_AT(LevelPattern& L) {
    product_rows(L.n_units, L.n_agg, L.AT_rp, L.AT_ci, L.AT_pp, L.AT_pa, L.AT_pt, [&](int64_t e, auto&& emit) {
        for (int32_t a = L.A_rp[e]; a < L.A_rp[e + 1]; ++a) {
            const int32_t c = L.A_ci[a];
            for (int32_t t = L.T_rp[c]; t < L.T_rp[c + 1]; ++t) emit(L.T_ci[t], a, t);
        }
    });
}

// A_{k+1} = T^T (A T): row I, block J = sum over units e with T(e,I), AT(e,J).
static void symbolic_C(LevelPattern& L) {
    product_rows(L.n_agg, L.n_agg, L.C_rp, L.C_ci, L.C_pp, L.C_pt, L.C_pu, [&](int64_t I, auto&& emit) {
        for (int32_t rr = L.R_rp[I]; rr < L.R_rp[I + 1]; ++rr) {
            const int32_t e = L.R_ci[rr], t = L.R_t[rr];
            for (int32_t u = L.AT_rp[e]; u < L.AT_rp[e + 1]; ++u) emit(L.AT_ci[u], t, u);
        }
    });
}

// M = R (D - omega A): row I, block c = sum over e with R(I,e), A(e,c).
void symbolic_M(LevelPattern& L) {
    if (L.M_done) return;
    product_rows(L.n_agg, L.n_units, L.M_rp, L.M_ci, L.M_pp, L.M_pr, L.M_pa, [&](int64_t I, auto&& emit) {
        for (int32_t rr = L.R_rp[I]; rr < L.R_rp[I + 1]; ++rr) {
            const int32_t e = L.R_ci[rr];
            for (int32_t a = L.A_rp[e]; a < L.A_rp[e + 1]; ++a) emit(L.A_ci[a], rr, a);
        }
    });
    L.M_done = true;
}

static void diag_positions(const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                           std::vector<int32_t>& diag, const char* what) {
    int64_t n = int64_t(rp.size()) - 1;
    diag.assign(n, -1);
    for (int64_t i = 0; i < n; ++i) {
        auto b = ci.begin() + rp[i], e = ci.begin() + rp[i + 1];
        auto it = std::lower_bound(b, e, int32_t(i));
        if (it == e || *it != i) fail(std::string(what) + ": missing diagonal block");
        diag[i] = int32_t(it - ci.begin());
    }
}

void build_plan(Plan& P, int64_t n_elem, const int32_t* row_ptr, const int32_t* col_idx, int64_t nnzb,
                int32_t n_levels, const int32_t* agg, bool hstar_smooth) {
    if (n_elem < 1 || !row_ptr || !col_idx || n_levels < 1) fail("plan: bad arguments");
    if (n_levels > 1 && !agg) fail("plan: aggregate hierarchy missing");
    if (n_elem >= (int64_t(1) << 31) || nnzb >= (int64_t(1) << 31)) fail("plan: sizes exceed int32 indexing");
    if (row_ptr[0] != 0 || row_ptr[n_elem] != nnzb) fail("plan: row_ptr does not span nnzb");
    for (int64_t e = 0; e < n_elem; ++e) {
        if (row_ptr[e + 1] < row_ptr[e]) fail("plan: row_ptr not monotone");
        for (int32_t a = row_ptr[e]; a < row_ptr[e + 1]; ++a) {
            if (col_idx[a] < 0 || col_idx[a] >= n_elem) fail("plan: column index out of range");
            if (a > row_ptr[e] && col_idx[a] <= col_idx[a - 1]) fail("plan: columns unsorted or duplicated");
        }
    }
    P.n_elem = n_elem;
    P.n_levels = n_levels;
    const int N = n_levels - 1;

    // per-level unit -> aggregate maps, nesting and density checks
    std::vector<std::vector<int32_t>> up(N);   // up[k]: level-k unit -> level-(k+1) aggregate
    std::vector<int64_t> nunits(n_levels);
    nunits[0] = n_elem;
    for (int k = 0; k < N; ++k) {
        const int32_t* a = agg + int64_t(k) * n_elem;
        int32_t mx = -1;
        for (int64_t e = 0; e < n_elem; ++e) {
            if (a[e] < 0) fail("plan: negative aggregate id");
            mx = std::max(mx, a[e]);
        }
        nunits[k + 1] = int64_t(mx) + 1;
        std::vector<int32_t>& u = up[k];
        u.assign(nunits[k], -1);
        std::vector<char> used(nunits[k + 1], 0);
        for (int64_t e = 0; e < n_elem; ++e) {
            int64_t unit = (k == 0) ? e : agg[int64_t(k - 1) * n_elem + e];
            if (u[unit] < 0) u[unit] = a[e];
            else if (u[unit] != a[e]) fail("plan: hierarchy is not nested");
            used[a[e]] = 1;
        }
        for (int64_t J = 0; J < nunits[k + 1]; ++J)
            if (!used[J]) fail("plan: aggregate ids are not dense");
        for (int64_t v = 0; v < nunits[k]; ++v)
            if (u[v] < 0) fail("plan: a unit has no aggregate");
        if (k > 0)
            for (int64_t v = 1; v < nunits[k]; ++v)
                if (u[v] < u[v - 1]) fail("plan: children of an aggregate must have consecutive ids");
    }

    // element renumbering: sort by (level-1 aggregate, element id)
    P.perm.resize(n_elem);
    std::iota(P.perm.begin(), P.perm.end(), 0);
    if (N > 0) {
        const int32_t* a1 = agg;
        std::stable_sort(P.perm.begin(), P.perm.end(), [&](int64_t x, int64_t y) { return a1[x] < a1[y]; });
    }
    P.iperm.resize(n_elem);
    for (int64_t i = 0; i < n_elem; ++i) P.iperm[P.perm[i]] = i;

    // level-0 pattern in internal order
    std::vector<int32_t> rp(n_elem + 1, 0), ci(nnzb);
    P.A0_src.resize(nnzb);
    {
        std::vector<std::pair<int32_t, int64_t>> row;
        for (int64_t u = 0; u < n_elem; ++u) {
            int64_t e = P.perm[u];
            row.clear();
            for (int32_t a = row_ptr[e]; a < row_ptr[e + 1]; ++a) row.push_back({int32_t(P.iperm[col_idx[a]]), a});
            std::sort(row.begin(), row.end());
            rp[u + 1] = rp[u] + int32_t(row.size());
            for (size_t j = 0; j < row.size(); ++j) {
                ci[rp[u] + j] = row[j].first;
                P.A0_src[rp[u] + j] = row[j].second;
            }
        }
    }

    P.lv.resize(N);
    for (int k = 0; k < N; ++k) {
        LevelPattern& L = P.lv[k];
        L.n_units = nunits[k];
        L.n_agg = nunits[k + 1];
        L.agg.resize(L.n_units);
        if (k == 0)
            for (int64_t u = 0; u < L.n_units; ++u) L.agg[u] = up[0][P.perm[u]];
        else
            L.agg = up[k];
        L.first_child.assign(L.n_agg + 1, 0);
        for (int64_t u = 0; u < L.n_units; ++u) L.first_child[L.agg[u] + 1]++;
        for (int64_t J = 0; J < L.n_agg; ++J) L.first_child[J + 1] += L.first_child[J];
        L.A_rp.swap(rp);
        L.A_ci.swap(ci);
        diag_positions(L.A_rp, L.A_ci, L.A_diag, k == 0 ? "A_0" : "A_k");
        L.replicated = L.n_agg == L.n_units;
        symbolic_T(L, L.replicated && !hstar_smooth);
        symbolic_R(L);
        symbolic_AT(L);
        symbolic_C(L);
        rp = L.C_rp;
        ci = L.C_ci;
    }
    P.AN_rp.swap(rp);
    P.AN_ci.swap(ci);
    diag_positions(P.AN_rp, P.AN_ci, P.AN_diag, "A_N");
}

}  // namespace amgdg
