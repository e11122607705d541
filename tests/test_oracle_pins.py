"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
generator outputs, closed forms from an eigendecomposition, brute-force dense
linear algebra, invariants the paper states (isometry of P~, R = T^T, symmetry
of the Galerkin operator and of the symmetric V-cycle) and special cases where
the method reduces to a direct solve.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import amg, krylov, rcb, rng
from workloads import configs, dg, mesh as meshes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense_D(Ad, nb):
    D = np.zeros_like(Ad)
    for u in range(Ad.shape[0] // nb):
        s = slice(u * nb, (u + 1) * nb)
        D[s, s] = Ad[s, s]
    return D


@pytest.fixture(scope="module")
def tiny():
    """2D SIPG p=1 on 8x8 split squares: 128 triangles, 384 dofs."""
    w = configs.poisson2d_split(nx=8, p=1, n_levels=3, bisections=2, r=2, nu=2)
    return w


# ---------------------------------------------------------------- generator

def test_splitmix64_published_vectors():
    lines = [l.split() for l in open(os.path.join(GOLD, "splitmix64.txt")) if not l.startswith("#")]
    seed, want = None, {}
    for l in lines:
        if l[0] == "seed":
            seed = int(l[1])
            want[seed] = []
        else:
            want[seed].append(int(l[0]))
    for s, vals in want.items():
        got = [int(v) for v in rng.splitmix64(s, len(vals))]
        assert got == vals


def test_uniform_range_and_normal_moments():
    u = rng.uniform_pm1(7, 200_000)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 3.0) < 0.01
    z = rng.normal(7, 200_000)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.02


# ---------------------------------------------------------------- hierarchy

def test_rcb_partition_nesting_and_sizes():
    m = meshes.jittered_delaunay(23, seed=3)
    cent = m.centroids()
    ne = len(cent)
    D = rcb.tree_depth(ne)
    for depth, perm, start in rcb.rcb_segments(cent):
        sizes = np.diff(start)
        assert sorted(perm) == list(range(ne))
        lo, hi = ne // 2 ** depth, -(-ne // 2 ** depth)
        big = sizes[sizes > 1]
        assert np.all((big >= lo) & (big <= hi)) or depth >= D - 1
    aggs, leaf = rcb.rcb_hierarchy(cent, 4, 2)
    # nesting: every level-k unit maps to exactly one level-(k+1) aggregate, ids dense
    for a in aggs:
        assert a.min() == 0 and len(np.unique(a)) == a.max() + 1
    # aggregates are contiguous ranges of the depth-first leaf order
    elem_levels = rcb.agg_of_elem_levels(aggs)
    for ea in elem_levels:
        seq = ea[leaf]
        assert np.all(np.diff(seq) >= 0)


def test_rcb_structured_counts():
    # 16x16 split squares, 3 levels of 8-way splits: 64 aggregates of 8, 8 of 64
    m = meshes.split_square(16)
    aggs, _ = rcb.rcb_hierarchy(m.centroids(), 3, 3)
    assert np.all(np.bincount(aggs[0]) == 8) and len(np.bincount(aggs[0])) == 64
    assert np.all(np.bincount(aggs[1]) == 8) and len(np.bincount(aggs[1])) == 8


def test_rcb_bisects_along_largest_extent():
    # points on a 4 x 2 lattice stretched in x: the first cut must split x
    pts = np.array([[x, y] for y in range(2) for x in range(4)], dtype=float) * [3.0, 1.0]
    seg = list(rcb.rcb_segments(pts))
    depth1_perm, depth1_start = seg[1][1], seg[1][2]
    left = set(depth1_perm[:depth1_start[1]])
    assert left == {0, 1, 4, 5}   # x in {0, 3}
    # ties on the key are broken by element id
    pts = np.zeros((4, 2))
    seg = list(rcb.rcb_segments(pts))
    assert list(seg[1][1]) == [0, 1, 2, 3]


# ---------------------------------------------------------------- smoother pieces

def test_block_inverse(tiny):
    A = tiny.A.to_scipy()
    D = amg.diag_blocks(A, A.shape[0] // 3, 3)
    Dinv = amg.block_inverse(D)
    assert np.abs(np.einsum("uij,ujk->uik", Dinv, D) - np.eye(3)).max() < 1e-12
    # diagonal blocks against a dense extraction
    Ad = A.toarray()
    assert np.array_equal(dense_D(Ad, 3)[:3, :3], D[0])


def _gen_eig(Ad, nb):
    """D^{-1}A = D^{-1/2} Q diag(lam) Q^T D^{1/2} for SPD A and block diagonal D."""
    D = dense_D(Ad, nb)
    Dh = sla.sqrtm(D).real
    Dmh = np.linalg.inv(Dh)
    lam, Q = np.linalg.eigh(Dmh @ Ad @ Dmh)
    return lam, Q, Dh, Dmh


def test_power_iteration_closed_form(tiny):
    A = tiny.A.to_scipy()
    Ad = A.toarray()
    nb = 3
    Dinv = amg.block_inverse(amg.diag_blocks(A, A.shape[0] // nb, nb))
    x0 = rng.uniform_pm1(3, A.shape[0])
    lam, Q, Dh, Dmh = _gen_eig(Ad, nb)

    def powk(k):
        return Dmh @ Q @ (lam ** k * (Q.T @ (Dh @ x0)))

    for q in (1, 3, 6):
        want = np.linalg.norm(powk(q + 1)) / np.linalg.norm(powk(q))
        got = amg.power_rho(A, Dinv, nb, q, x0)
        assert abs(got - want) < 1e-12 * want
    assert amg.power_rho(A, Dinv, nb, 3, x0) <= lam.max() * (1 + 1e-12)


def test_power_iteration_1d_laplacian():
    # 1D FD Laplacian, 1x1 blocks: rho(D^-1 A) = 1 + cos(pi h); omega -> 2/3 as q grows
    import scipy.sparse as sp
    n = 31
    h = 1.0 / (n + 1)
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    Dinv = np.full((n, 1, 1), 0.5)
    rho = 1 + math.cos(math.pi * h)
    x0 = rng.uniform_pm1(11, n)
    assert amg.power_rho(A, Dinv, 1, 3, x0) <= rho + 1e-12
    est = amg.power_rho(A, Dinv, 1, 4000, x0)
    assert abs(est - rho) < 1e-6
    assert abs(amg.omega_from_rho(2.0) - 2.0 / 3.0) < 1e-15


def test_relaxation_count_and_iterate_closed_form(tiny):
    A = tiny.A.to_scipy()
    Ad = A.toarray()
    nb = 3
    Dinv = amg.block_inverse(amg.diag_blocks(A, A.shape[0] // nb, nb))
    lam, Q, Dh, Dmh = _gen_eig(Ad, nb)
    omega, gamma = 0.7, 0.03
    x0 = np.random.default_rng(2).standard_normal(A.shape[0])
    c = Q.T @ (Dh @ x0)

    def it(m):  # S^m x0 with S = I - omega D^-1 A
        return Dmh @ Q @ ((1 - omega * lam) ** m * c)

    m_want = next(m for m in range(1, 1000)
                  if np.linalg.norm(it(m - 1)) / np.linalg.norm(it(m)) < 1 + gamma)
    x, m_got = amg.relax_candidate(A, Dinv, nb, omega, x0.copy(), gamma, 100)
    assert m_got == m_want
    assert np.linalg.norm(x - it(m_got)) < 1e-11 * np.linalg.norm(x)
    # the cap binds
    _, m_cap = amg.relax_candidate(A, Dinv, nb, omega, x0.copy(), -1.0, 7)
    assert m_cap == 7


# ---------------------------------------------------------------- P~, T, R, A_{k+1}

@pytest.fixture(scope="module")
def tiny_h(tiny):
    A = tiny.A.to_scipy()
    aggs, _ = rcb.rcb_hierarchy(tiny.centroids, 3, 2)
    H = amg.setup(A, 3, aggs, tiny.params, tiny.B1)
    return tiny, A, aggs, H


def test_tentative_prolongator_isometry_and_reproduction(tiny_h):
    _, A, aggs, H = tiny_h
    for L in H.levels[:-1]:
        P = L.P.toarray()
        assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12          # isometry (eq:splitB)
        # s = r here, so P P^T reproduces the candidates exactly on each aggregate
        assert L.s == L.B.shape[1]
        assert np.abs(P @ (P.T @ L.B) - L.B).max() < 1e-11 * np.abs(L.B).max()
        # singular values: sqrt of the eigenvalues of the Gram matrix, per aggregate
        order = np.argsort(L.agg, kind="stable")
        J = 0
        units = order[L.agg[order] == J]
        dofs = (units[:, None] * L.nb + np.arange(L.nb)).ravel()
        M = L.B[dofs]
        ev = np.sqrt(np.sort(np.linalg.eigvalsh(M.T @ M))[::-1])
        assert np.allclose(L.sv[J], ev, rtol=1e-8)
        # canonical sign: largest-magnitude entry of each column positive
        cols = P[dofs][:, :L.s]
        piv = cols[np.argmax(np.abs(cols), axis=0), np.arange(L.s)]
        assert np.all(piv > 0)


def test_smoothed_prolongator_and_galerkin_dense(tiny_h):
    _, A, _, H = tiny_h
    L = H.levels[0]
    Ad = A.toarray()
    Dinv_d = np.linalg.inv(dense_D(Ad, L.nb))
    T = (np.eye(Ad.shape[0]) - L.omega * Dinv_d @ Ad) @ L.P.toarray()
    assert np.abs(L.T.toarray() - T).max() < 1e-12 * np.abs(T).max()
    assert np.array_equal(L.R.toarray(), L.T.toarray().T)
    Ac = T.T @ Ad @ T
    A1 = H.levels[1].A.toarray()
    assert np.abs(A1 - Ac).max() < 1e-12 * np.abs(Ac).max()
    assert np.abs(A1 - A1.T).max() < 1e-13 * np.abs(A1).max()          # symmetric fluxes
    np.linalg.cholesky(A1)                                               # SPD


def test_block_patterns_match_numeric_support(tiny_h):
    w, A, aggs, H = tiny_h
    pats = amg.block_patterns(w.A.row_ptr, w.A.col_idx, aggs)
    for k, L in enumerate(H.levels[:-1]):
        s, nb = L.s, L.nb
        Tb = abs(L.T).tobsr(blocksize=(nb, s))
        Tb.sort_indices()
        # numeric support is contained in the structural pattern
        S = set(zip(np.repeat(np.arange(len(pats[k]["T_ptr"]) - 1), np.diff(pats[k]["T_ptr"])), pats[k]["T_idx"]))
        rows = np.repeat(np.arange(Tb.shape[0] // nb), np.diff(Tb.indptr))
        nz = [(r, c) for r, c, b in zip(rows, Tb.indices, Tb.data) if np.any(b != 0)]
        assert set(nz) <= S
        assert len(nz) == len(S)     # generic data: no cancellation to exact zero


def test_two_grid_error_propagator(tiny):
    """E = I - V A equals S^nu (I - T A_c^{-1} T^T A) S^nu for a two-level cycle."""
    w = tiny
    A = w.A.to_scipy()
    Ad = A.toarray()
    n = Ad.shape[0]
    aggs, _ = rcb.rcb_hierarchy(w.centroids, 2, 2)
    H = amg.setup(A, 3, aggs, dataclasses.replace(w.params, n_levels=2), w.B1)
    L = H.levels[0]
    V = np.stack([amg.vcycle(H, e) for e in np.eye(n)], axis=1)
    S = np.eye(n) - L.omega * np.linalg.inv(dense_D(Ad, 3)) @ Ad
    T = L.T.toarray()
    CG = np.eye(n) - T @ np.linalg.solve(T.T @ Ad @ T, T.T @ Ad)
    nu = w.params.t_pre
    E = np.linalg.matrix_power(S, nu) @ CG @ np.linalg.matrix_power(S, nu)
    assert np.abs((np.eye(n) - V @ Ad) - E).max() < 1e-10


# ---------------------------------------------------------------- V-cycle

def test_vcycle_linear_and_symmetric(tiny_h):
    w, A, _, H = tiny_h
    g = np.random.default_rng(9)
    b1, b2 = g.standard_normal(A.shape[0]), g.standard_normal(A.shape[0])
    v = amg.vcycle(H, 2.5 * b1 + b2)
    assert np.linalg.norm(v - (2.5 * amg.vcycle(H, b1) + amg.vcycle(H, b2))) < 1e-12 * np.linalg.norm(v)
    lhs, rhs = amg.vcycle(H, b1) @ b2, b1 @ amg.vcycle(H, b2)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-14
    # positive definite on random vectors
    assert amg.vcycle(H, b1) @ b1 > 0


def test_vcycle_exact_when_coarse_space_is_everything(tiny):
    """Singleton aggregates and s = nb: T is square and invertible, so the coarse
    correction T (T^T A T)^{-1} T^T is A^{-1} and one cycle solves exactly.
    Singleton aggregates are h*-steps (eq:sik): delta = 0 keeps every nonzero
    singular value, i.e. s = nb."""
    w = tiny
    A = w.A.to_scipy()
    ne = A.shape[0] // 3
    prm = dataclasses.replace(w.params, n_levels=2, r=3, n_cut=1.0, delta=0.0)
    H = amg.setup(A, 3, [np.arange(ne, dtype=np.int32)], prm,
                  np.random.default_rng(2).standard_normal((A.shape[0], 3)))
    b = np.random.default_rng(4).standard_normal(A.shape[0])
    x = sla.solve(A.toarray(), b)
    assert np.linalg.norm(amg.vcycle(H, b) - x) < 1e-11 * np.linalg.norm(x)


def test_vcycle_fp32_close_to_fp64(tiny_h):
    _, A, _, H = tiny_h
    b = np.random.default_rng(5).standard_normal(A.shape[0])
    v64 = amg.vcycle(H, b)
    v32 = amg.vcycle_fp32(H, amg.to_fp32(H), b).astype(np.float64)
    rel = np.linalg.norm(v32 - v64) / np.linalg.norm(v64)
    assert 0 < rel < 1e-4


# ---------------------------------------------------------------- outer iterations

def test_pcg_exact_preconditioner_one_iteration(tiny):
    A = tiny.A.to_scipy()
    Ad = A.toarray()
    b = tiny.b
    x, it, _ = krylov.pcg(A, b, lambda r: sla.solve(Ad, r), 1e-10, 10)
    assert it == 1
    assert np.linalg.norm(x - sla.solve(Ad, b)) < 1e-10 * np.linalg.norm(x)


def test_fgmres_minimises_over_krylov_space():
    m = meshes.jittered_delaunay(9, seed=1)
    Ab = dg.assemble_ldg_upwind(m, 1, np.array([np.cos(0.3), np.sin(0.3)]), 1e-2)
    A = Ab.to_scipy()
    Ad = A.toarray()
    n = Ad.shape[0]
    b = np.random.default_rng(1).uniform(-1, 1, n)
    Mmat = np.linalg.inv(dense_D(Ad, Ab.nb))   # a fixed linear preconditioner
    for j in (3, 8):
        x, it, _ = krylov.fgmres(A, b, lambda v: Mmat @ v, 1e-30, j, j)
        assert it == j
        K = [Mmat @ b]
        for _ in range(j - 1):
            K.append(Mmat @ (Ad @ K[-1]))
        Z = np.linalg.qr(np.stack(K, 1))[0]
        y = np.linalg.lstsq(Ad @ Z, b, rcond=None)[0]
        best = np.linalg.norm(b - Ad @ Z @ y)
        assert abs(np.linalg.norm(b - Ad @ x) - best) < 1e-9 * np.linalg.norm(b)


def test_full_solve_against_direct():
    w = configs.poisson2d_split()          # 1,536 dofs
    A = w.A.to_scipy()
    Ad = A.toarray()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
    H = amg.setup(A, w.A.nb, aggs, w.params, w.B1)
    xs = sla.solve(Ad, w.b)
    kappa = np.linalg.cond(Ad)
    for solver in (lambda M: krylov.pcg(A, w.b, M, 1e-8, 2000),
                   lambda M: krylov.fcg(A, w.b, M, 1e-8, 2000)):
        x, it, _ = solver(lambda r: amg.vcycle(H, r))
        assert np.linalg.norm(w.b - A @ x) <= 1e-8 * np.linalg.norm(w.b)
        assert np.linalg.norm(x - xs) <= kappa * 1e-8 * np.linalg.norm(xs)
    M32 = amg.to_fp32(H)
    x, it, _ = krylov.fgmres(A, w.b, lambda r: amg.vcycle_fp32(H, M32, r).astype(np.float64), 1e-8, 400, 2000)
    assert np.linalg.norm(w.b - A @ x) <= 1e-8 * np.linalg.norm(w.b)


# ---------------------------------------------------------------- Algorithm 2 as a solver

def test_stationary_exact_preconditioner_one_step(tiny):
    """With M = A^{-1} the correction x + M(b - A x) is the solution after one step."""
    A = tiny.A.to_scipy()
    Ad = A.toarray()
    x, it, hist = krylov.stationary(A, tiny.b, lambda r: sla.solve(Ad, r), 1e-12, 10)
    assert it == 1 and len(hist) == 1
    xs = sla.solve(Ad, tiny.b)
    assert np.linalg.norm(x - xs) < 1e-12 * np.linalg.norm(xs)


def test_stationary_iterates_are_the_neumann_partial_sums(tiny):
    """For a fixed linear M, iterate k from x = 0 is sum_{j<k} (I - MA)^j M b
    (formed densely), and the solver stops at the first k whose true relative
    residual meets the tolerance, not one step earlier or later."""
    A = tiny.A.to_scipy()
    Ad = A.toarray()
    n = Ad.shape[0]
    Mm = 0.7 * np.linalg.inv(dense_D(Ad, 3))          # a fixed linear preconditioner
    b = tiny.b
    E = np.eye(n) - Mm @ Ad
    sums, term, acc = [], Mm @ b, np.zeros(n)
    for _ in range(8):
        acc = acc + term
        sums.append(acc.copy())
        term = E @ term
    for k in (1, 2, 5, 8):
        x, it, hist = krylov.stationary(A, b, lambda r: Mm @ r, 0.0, k)
        assert it == k and len(hist) == k
        assert np.linalg.norm(x - sums[k - 1]) < 1e-12 * np.linalg.norm(sums[k - 1])
    res = [np.linalg.norm(b - Ad @ s) / np.linalg.norm(b) for s in sums]
    assert all(res[j + 1] < res[j] for j in range(len(res) - 1))
    kstar = 5
    tol = math.sqrt(res[kstar - 2] * res[kstar - 1])   # between the residuals of steps 4 and 5
    _, it, _ = krylov.stationary(A, b, lambda r: Mm @ r, tol, 100)
    assert it == kstar


# ---------------------------------------------------------------- eq:sik truncation (s < r)

def test_coarse_size_rounding_and_caps():
    """eq:sik h-step: |A_J| / n_cut read as the ceiling, capped by the rank
    min(|A_J|, r) that the |A_J| x r candidate block can supply."""
    assert amg.coarse_size(12, 5.0, 6) == 3          # ceil(2.4); the floor would give 2
    assert amg.coarse_size(12, 3.0, 6) == 4          # exact quotient
    assert amg.coarse_size(12, 5.0, 2) == 2          # r binds
    assert amg.coarse_size(2, 1.0, 6) == 2           # |A_J| binds
    assert amg.coarse_size(40, 3.0, 40) == 14        # the oversampled 2D case: ceil(13.3)


def test_truncated_prolongator_spans_the_leading_singular_subspace(tiny):
    """s_J < r: on each aggregate the kept columns of P~ span the dominant
    s_J-dimensional left singular subspace of B^k[A_J, :], i.e. P~_J P~_J^T is
    the projector onto the top s_J eigenvectors of B_J B_J^T (dense eigh)."""
    w = tiny
    A = w.A.to_scipy()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, 2, 2)
    assert np.all(np.bincount(aggs[0]) == 4)               # |A_J| = 12 dofs each
    r, n_cut = 6, 5.0
    prm = dataclasses.replace(w.params, n_levels=2, r=r, n_cut=n_cut)
    B1 = np.random.default_rng(2).standard_normal((A.shape[0], r))
    H = amg.setup(A, 3, aggs, prm, B1)
    L = H.levels[0]
    assert L.s == 3 and L.s < r
    P = L.P.toarray()
    assert P.shape[1] == 3 * (aggs[0].max() + 1)
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12
    order = np.argsort(L.agg, kind="stable")
    for J in range(int(L.agg.max()) + 1):
        units = order[L.agg[order] == J]
        dofs = (units[:, None] * 3 + np.arange(3)).ravel()
        BJ = L.B[dofs]
        lam, Q = np.linalg.eigh(BJ @ BJ.T)
        assert lam[-3] > 1e-6 * lam[-1] and lam[-4] < (1 - 1e-3) * lam[-3]   # a gap to truncate at
        proj = Q[:, -3:] @ Q[:, -3:].T
        PJ = P[dofs][:, 3 * J:3 * J + 3]
        assert np.abs(PJ @ PJ.T - proj).max() < 1e-10
        # every other column of P~ is zero on these rows
        assert np.abs(np.delete(P[dofs], np.s_[3 * J:3 * J + 3], axis=1)).max() == 0.0
        # singular values: the square roots of the Gram eigenvalues, descending
        assert np.allclose(L.sv[J], np.sqrt(np.clip(lam[::-1][:r], 0, None)), rtol=1e-8, atol=1e-12 * np.sqrt(lam[-1]))


# ---------------------------------------------------------------- convergence under refinement

@pytest.mark.slow
def test_convergence_factor_near_constant_under_refinement():
    """The paper's own problem and setup (Section 5.1: Q1 LDG on 2^M hexahedra
    per direction, V(3,3), r = the median dofs per level-1 aggregate = 64,
    n_cut = 6, tolerance 1e-7 from zero): the average convergence factor of
    multigrid as a solver and as the CG preconditioner stays near-constant as
    the mesh is refined (bound: factor <= 0.35, growth <= 0.1 per refinement),
    and the pCG counts are the paper's (6 at M = 3, 7 at M = 4) within one."""
    fac_cg, fac_st, its_cg = [], [], []
    for M in (2, 3, 4):
        w = configs.poisson3d_hex(M=M, p=1, flux="ldg", r=64)
        A = w.A.to_scipy()
        aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
        H = amg.setup(A, w.A.nb, aggs, w.params, w.B1)
        V = lambda v: amg.vcycle(H, v)
        _, it, hist = krylov.pcg(A, w.b, V, 1e-7, 200)
        _, its, hs = krylov.stationary(A, w.b, V, 1e-7, 200)
        assert hist[-1] <= 1e-7 and hs[-1] <= 1e-7
        fac_cg.append(hist[-1] ** (1.0 / it))
        fac_st.append(hs[-1] ** (1.0 / its))
        its_cg.append(it)
    for fac in (fac_cg, fac_st):
        assert max(fac) <= 0.35, fac
        assert all(fac[j + 1] - fac[j] <= 0.1 for j in range(len(fac) - 1)), fac
    assert abs(its_cg[1] - 6) <= 1 and abs(its_cg[2] - 7) <= 1, its_cg


# ---------------------------------------------------------------- units of unequal size (eq:sik per aggregate)

def test_block_diagonal_of_unequal_units():
    """D_k of a level whose units differ in size: the diagonal blocks equal a
    dense extraction, their inverses invert them, and applying them equals the
    dense block-diagonal product."""
    g = np.random.default_rng(12)
    sizes = np.array([3, 4, 3, 5, 4, 4, 2, 3])
    n = sizes.sum()
    X = g.standard_normal((n, n))
    Ad = X @ X.T + n * np.eye(n)
    import scipy.sparse as sp
    D = amg.BlockDiag.from_matrix(sp.csr_matrix(Ad), sizes)
    Dinv = D.inverse()
    offs = np.concatenate([[0], np.cumsum(sizes)])
    Dd = np.zeros_like(Ad)
    for u in range(len(sizes)):
        s = slice(offs[u], offs[u + 1])
        Dd[s, s] = Ad[s, s]
    assert np.array_equal(D.to_csr().toarray(), Dd)
    assert np.abs(Dinv.to_csr().toarray() @ Dd - np.eye(n)).max() < 1e-13
    x = g.standard_normal((n, 3))
    assert np.abs(Dinv.apply(x) - np.linalg.inv(Dd) @ x).max() < 1e-13
    assert np.abs(Dinv.apply(x[:, 0]) - np.linalg.inv(Dd) @ x[:, 0]).max() < 1e-13


@pytest.fixture(scope="module")
def mixed_sizes():
    """2D SIPG p=1 on 7x7 split squares (98 triangles): 4-way RCB gives level-1
    aggregates of 3 and 4 elements (9 and 12 dofs), so eq:sik with n_cut = 3
    and r = 6 keeps s_J = 3 or 4 coarse dofs per aggregate."""
    w = configs.poisson2d_split(nx=7, p=1, n_levels=3, bisections=2, r=6, nu=2)
    A = w.A.to_scipy()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, 3, 2)
    H = amg.setup(A, 3, aggs, w.params, w.B1)
    return w, A, aggs, H


def test_unequal_coarse_blocks_follow_eq_sik(mixed_sizes):
    w, A, aggs, H = mixed_sizes
    L = H.levels[0]
    counts = np.bincount(aggs[0])
    assert set(counts) == {3, 4}
    want = np.array([amg.coarse_size(3 * c, 3.0, 6) for c in counts])
    assert np.array_equal(L.s_agg, want) and set(want) == {3, 4}
    assert np.array_equal(H.levels[1].sizes, want)
    P = L.P.toarray()
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12
    coffs = np.concatenate([[0], np.cumsum(L.s_agg)])
    order = np.argsort(L.agg, kind="stable")
    for J in range(len(counts)):
        units = order[L.agg[order] == J]
        dofs = (units[:, None] * 3 + np.arange(3)).ravel()
        BJ = L.B[dofs]
        sJ = int(L.s_agg[J])
        lam, Q = np.linalg.eigh(BJ @ BJ.T)
        proj = Q[:, -sJ:] @ Q[:, -sJ:].T
        cols = slice(coffs[J], coffs[J + 1])
        assert np.abs(P[dofs][:, cols] @ P[dofs][:, cols].T - proj).max() < 1e-10
        others = np.ones(P.shape[1], bool)
        others[cols] = False
        assert np.abs(P[dofs][:, others]).max() == 0.0


def test_unequal_coarse_blocks_operators_dense(mixed_sizes):
    """T, R and A_1 over coarse units of unequal size against dense algebra,
    level 1's block-Jacobi diagonal taken per unit size, and the two-grid error
    propagator S^nu (I - T A_c^{-1} T^T A) S^nu of the cycle."""
    w, A, aggs, H = mixed_sizes
    Ad = A.toarray()
    L0, L1 = H.levels[0], H.levels[1]
    Dinv_d = np.linalg.inv(dense_D(Ad, 3))
    T = (np.eye(Ad.shape[0]) - L0.omega * Dinv_d @ Ad) @ L0.P.toarray()
    assert np.abs(L0.T.toarray() - T).max() < 1e-12 * np.abs(T).max()
    assert np.array_equal(L0.R.toarray(), L0.T.toarray().T)
    A1 = T.T @ Ad @ T
    assert np.abs(L1.A.toarray() - A1).max() < 1e-12 * np.abs(A1).max()
    offs = np.concatenate([[0], np.cumsum(L1.sizes)])
    D1 = np.zeros_like(A1)
    for u in range(len(L1.sizes)):
        s = slice(offs[u], offs[u + 1])
        D1[s, s] = A1[s, s]
    assert np.abs(L1.Dinv_bd.to_csr().toarray() - np.linalg.inv(D1)).max() < 1e-10 * np.abs(np.linalg.inv(D1)).max()
    # a two-level cycle on these operators
    H2 = amg.setup(A, 3, aggs[:1], dataclasses.replace(w.params, n_levels=2), w.B1)
    n = Ad.shape[0]
    V = np.stack([amg.vcycle(H2, e) for e in np.eye(n)], axis=1)
    S = np.eye(n) - H2.levels[0].omega * Dinv_d @ Ad
    T2 = H2.levels[0].T.toarray()
    CG = np.eye(n) - T2 @ np.linalg.solve(T2.T @ Ad @ T2, T2.T @ Ad)
    nu = w.params.t_pre
    E = np.linalg.matrix_power(S, nu) @ CG @ np.linalg.matrix_power(S, nu)
    assert np.abs((np.eye(n) - V @ Ad) - E).max() < 1e-10
    # the three-level cycle stays linear and symmetric
    g = np.random.default_rng(9)
    b1, b2 = g.standard_normal(n), g.standard_normal(n)
    v = amg.vcycle(H, 2.5 * b1 + b2)
    assert np.linalg.norm(v - (2.5 * amg.vcycle(H, b1) + amg.vcycle(H, b2))) < 1e-12 * np.linalg.norm(v)
    assert abs(amg.vcycle(H, b1) @ b2 - b1 @ amg.vcycle(H, b2)) < 1e-12 * abs(amg.vcycle(H, b1) @ b2)


# ---------------------------------------------------------------- h*-step (eq:sik, second case)

def test_hstar_step_keeps_singular_values_above_delta(tiny):
    """A level whose aggregates are its own units (Algorithm 5's replicated
    level): each element keeps the left singular vectors of its candidate
    block whose singular values exceed delta times the largest, counted here
    from the eigenvalues of M M^T, and P~ is block diagonal per element."""
    w = tiny
    A = w.A.to_scipy()
    ne = A.shape[0] // 3
    r = 8
    B1 = np.random.default_rng(2).standard_normal((A.shape[0], r))
    prm0 = dataclasses.replace(w.params, n_levels=2, r=r)
    H0 = amg.setup(A, 3, [np.arange(ne, dtype=np.int32)], dataclasses.replace(prm0, delta=0.0), B1)
    B = H0.levels[0].B
    ratios = []
    for e in range(ne):
        ev = np.sqrt(np.clip(np.linalg.eigvalsh(B[3 * e:3 * e + 3] @ B[3 * e:3 * e + 3].T)[::-1], 0, None))
        ratios.append(ev / ev[0])
    delta = float(np.median([rr[1] for rr in ratios]))          # splits the elements between s = 1 and s >= 2
    H = amg.setup(A, 3, [np.arange(ne, dtype=np.int32)], dataclasses.replace(prm0, delta=delta), B1)
    L = H.levels[0]
    want = np.array([int(np.count_nonzero(rr > delta)) for rr in ratios])
    assert np.array_equal(L.s_agg, want) and len(set(want)) >= 2
    P = L.P.toarray()
    coffs = np.concatenate([[0], np.cumsum(L.s_agg)])
    for e in range(ne):
        rows = slice(3 * e, 3 * e + 3)
        Pe = P[rows, coffs[e]:coffs[e + 1]]
        M = B[rows]
        lam, Q = np.linalg.eigh(M @ M.T)
        s = int(want[e])
        assert np.abs(Pe @ Pe.T - Q[:, -s:] @ Q[:, -s:].T).max() < 1e-10
        assert np.abs(np.delete(P[rows], np.s_[coffs[e]:coffs[e + 1]], axis=1)).max() == 0.0
