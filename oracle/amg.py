"""Geometric alpha-SA setup and V-cycle, FP64 (oracle side).

Follows Algorithm 5 (Section 4.5) with the index garbles of its listing read as
k = 0..N-1, T^k_{k+1} and A_{k+1} = R A_k T, and the V-cycle of Algorithm 2.
Plain NumPy/SciPy: sparse matrices at dof level, dense diagonal blocks, LAPACK
SVD and LU.  Level k has ``nunits`` units (elements at level 0, aggregates at
k >= 1); unit u owns the dofs [offs[u], offs[u+1]) of that level, nb dofs each
at level 0 and s_J (eq:sik, chosen per aggregate) on coarse levels.
"""
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .rng import uniform_pm1


@dataclass
class Level:
    A: sp.csr_matrix
    nb: int                       # dofs per unit when all units have the same size, else 0
    nunits: int
    sizes: np.ndarray = None      # dofs of each unit
    Dinv: np.ndarray = None       # (nunits, nb, nb) when the sizes are uniform
    Dinv_bd: "BlockDiag" = None   # D_k^{-1} for any sizes
    omega: float = float("nan")
    rho: float = float("nan")
    B_in: np.ndarray = None       # candidates before relaxation
    B: np.ndarray = None          # relaxed candidates
    sweeps: np.ndarray = None
    agg: np.ndarray = None        # unit -> level-(k+1) aggregate
    s: int = 0                    # largest coarse block size s_J of the level
    s_agg: np.ndarray = None      # s_J of every level-(k+1) aggregate
    sv: list = field(default_factory=list)
    P: sp.csr_matrix = None
    T: sp.csr_matrix = None
    R: sp.csr_matrix = None


@dataclass
class Hierarchy:
    levels: list
    lu: tuple
    t_pre: int
    t_post: int


# --------------------------------------------------------------------------
# setup steps
# --------------------------------------------------------------------------

def diag_blocks(A, nunits, nb):
    """D_k: the nb x nb diagonal blocks of A_k (block Jacobi, Section 4.4 item 2)."""
    Ab = A.tocsr().tobsr(blocksize=(nb, nb))
    Ab.sort_indices()
    rows = np.repeat(np.arange(nunits), np.diff(Ab.indptr))
    on_diag = Ab.indices == rows
    D = np.zeros((nunits, nb, nb))
    D[rows[on_diag]] = Ab.data[on_diag]
    return D


def block_inverse(D):
    """D_k^{-1} block by block (LAPACK LU with partial pivoting)."""
    return np.linalg.inv(D)


def apply_blockdiag(Binv, x, nb):
    """y = blockdiag(Binv) x for x of shape (n,) or (n, m)."""
    nun = Binv.shape[0]
    if x.ndim == 1:
        return np.einsum("uij,uj->ui", Binv, x.reshape(nun, nb)).ravel()
    m = x.shape[1]
    return np.einsum("uij,ujm->uim", Binv, x.reshape(nun, nb, m)).reshape(-1, m)


class BlockDiag:
    """A block-diagonal matrix with one dense square block per unit, unit u
    owning the dofs [offs[u], offs[u+1]) (D_k of block Jacobi, Section 4.4;
    after eq:sik the units of a coarse level may differ in size).  Units of
    equal size are held together as one (count, s, s) array."""

    def __init__(self, sizes, groups):
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.offs = np.concatenate([[0], np.cumsum(self.sizes)])
        self.groups = groups          # list of (s, units, dof index (count, s), blocks (count, s, s))

    @staticmethod
    def index_groups(sizes):
        sizes = np.asarray(sizes, dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        out = []
        for sz in np.unique(sizes):
            units = np.nonzero(sizes == sz)[0]
            out.append((int(sz), units, offs[units][:, None] + np.arange(sz)[None, :]))
        return out

    @classmethod
    def from_matrix(cls, A, sizes):
        """The diagonal blocks of A."""
        A = A.tocsr()
        groups = []
        offs = np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))])
        for sz, units, idx in cls.index_groups(sizes):
            sub = A[idx.ravel(), :].tocoo()
            u_loc = sub.row // sz
            i_loc = sub.row % sz
            j_loc = sub.col - offs[units[u_loc]]
            keep = (j_loc >= 0) & (j_loc < sz)
            D = np.zeros((len(units), sz, sz))
            np.add.at(D, (u_loc[keep], i_loc[keep], j_loc[keep]), sub.data[keep])
            groups.append((sz, units, idx, D))
        return cls(sizes, groups)

    def inverse(self):
        """Block by block (LAPACK LU with partial pivoting)."""
        return BlockDiag(self.sizes, [(sz, u, idx, np.linalg.inv(D)) for sz, u, idx, D in self.groups])

    def astype(self, dt):
        return BlockDiag(self.sizes, [(sz, u, idx, D.astype(dt)) for sz, u, idx, D in self.groups])

    def apply(self, x):
        """y = blockdiag(D_u) x for x of shape (n,) or (n, m)."""
        if len(self.groups) == 1:                   # equal sizes: units in order
            D = self.groups[0][3]
            return apply_blockdiag(D, x, D.shape[1])
        y = np.zeros(x.shape, dtype=np.result_type(x.dtype, self.groups[0][3].dtype))
        for sz, units, idx, D in self.groups:
            if x.ndim == 1:
                y[idx] = np.einsum("uij,uj->ui", D, x[idx])
            else:
                y[idx] = np.einsum("uij,ujm->uim", D, x[idx])
        return y

    def to_csr(self):
        rows, cols, vals = [], [], []
        for sz, units, idx, D in self.groups:
            rows.append(np.repeat(idx, sz, axis=1).ravel())
            cols.append(np.tile(idx, (1, sz)).ravel())
            vals.append(D.ravel())
        n = int(self.offs[-1])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    def uniform_array(self):
        """(nunits, nb, nb) when every unit has the same size, else None."""
        if len(self.groups) != 1:
            return None
        return self.groups[0][3]


def _apply_dinv(Dinv, x, nb):
    return Dinv.apply(x) if isinstance(Dinv, BlockDiag) else apply_blockdiag(Dinv, x, nb)


def power_rho(A, Dinv, nb, q, x0):
    """Algorithm 4: estimate rho(D^{-1} A) with q power steps from a unit vector.

    Reading: the listing's 'x = Ax' is the level operator A_k."""
    x = x0 / np.linalg.norm(x0)
    for _ in range(q):
        x = A @ x
        x = _apply_dinv(Dinv, x, nb)
        x = x / np.linalg.norm(x)
    return float(np.linalg.norm(_apply_dinv(Dinv, A @ x, nb)))


def omega_from_rho(rho):
    """eq:omega: omega_k = (4/3) / rho_k."""
    return (4.0 / 3.0) / rho


def relax_candidate(A, Dinv, nb, omega, x, gamma, relax_max):
    """eq:bsmooth: smooth A_k x = 0 with x <- x + omega D^{-1}(0 - A x) until the
    norm ratio of consecutive iterates ||x^(m)|| / ||x^(m+1)|| drops below 1+gamma.

    Readings: 2-norm; at least one sweep; at most relax_max sweeps; the iterate
    that passes the test is returned (no normalisation).  Returns (x, sweeps)."""
    m = 0
    while True:
        y = x - omega * _apply_dinv(Dinv, A @ x, nb)
        m += 1
        stop = np.linalg.norm(x) / np.linalg.norm(y) < 1.0 + gamma
        x = y
        if stop or m >= relax_max:
            return x, m


def canonical_sign(U):
    """Flip each column so that its entry of largest magnitude is positive
    (ties: the lowest row).  Fixes the sign freedom of the SVD."""
    idx = np.argmax(np.abs(U), axis=-2)
    piv = np.take_along_axis(U, idx[..., None, :], axis=-2)
    return U * np.where(piv < 0, -1.0, 1.0)


def coarse_size(n_rows, n_cut, r):
    """eq:sik, h-step: |A_J| / n_cut vectors, read as ceil and capped by the rank
    the SVD of the |A_J| x r block can supply."""
    return min(math.ceil(n_rows / n_cut), n_rows, r)


def hstar_size(svals, delta):
    """eq:sik, h*-step (an aggregate that equals its only child): the number of
    singular values above delta times the largest."""
    sv = np.asarray(svals)
    return int(np.count_nonzero(sv > delta * sv[0])) if len(sv) and sv[0] > 0 else 0


def tentative_prolongator(B, agg, sizes, n_cut, delta=1e-3):
    """eq:splitB_dg + eq:sik: per aggregate J, SVD of B[rows of J, :] (the dofs
    of J's children, children in increasing unit id) and P_J = the leading s_J
    left singular vectors (canonical sign).  s_J follows eq:sik per aggregate:
    the h-step count (coarse_size) when J has several children, the h*-step
    count (hstar_size, threshold delta) when J equals its only child.

    sizes: dofs of every unit of this level (an int for equal sizes).
    Returns (P as csr, s_J per aggregate, singular values per aggregate padded
    with zeros to r)."""
    r = B.shape[1]
    agg = np.asarray(agg, dtype=np.int64)
    nunits = len(agg)
    sizes = np.full(nunits, sizes, dtype=np.int64) if np.isscalar(sizes) else np.asarray(sizes, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    nagg = int(agg.max()) + 1
    order = np.argsort(agg, kind="stable")      # children of each J in increasing unit id
    counts = np.bincount(agg, minlength=nagg)
    su = sizes[order]
    dof_order = np.repeat(offs[order], su) + (np.arange(su.sum()) - np.repeat(np.cumsum(su) - su, su))
    nrows = np.bincount(agg, weights=sizes, minlength=nagg).astype(np.int64)
    dstart = np.concatenate([[0], np.cumsum(nrows)])
    s_agg = np.zeros(nagg, dtype=np.int64)
    svals = [None] * nagg
    Us = []
    for c in np.unique(nrows):
        Js = np.nonzero(nrows == c)[0]
        dofs = dof_order[dstart[Js][:, None] + np.arange(c)[None, :]]          # (G, c)
        U, S, _ = np.linalg.svd(B[dofs], full_matrices=False)
        U = canonical_sign(U)
        for g, J in enumerate(Js):
            s_agg[J] = hstar_size(S[g], delta) if counts[J] == 1 else coarse_size(int(c), n_cut, r)
            svals[J] = np.concatenate([S[g], np.zeros(r - len(S[g]))])
        Us.append((Js, dofs, U))
    coffs = np.concatenate([[0], np.cumsum(s_agg)])
    rows_P, cols_P, vals_P = [], [], []
    for Js, dofs, U in Us:
        sj = s_agg[Js]
        for l in range(int(sj.max())):
            sel = sj > l
            rows_P.append(dofs[sel].ravel())
            cols_P.append(np.repeat(coffs[Js[sel]] + l, dofs.shape[1]))
            vals_P.append(U[sel, :, l].ravel())
    P = sp.csr_matrix((np.concatenate(vals_P), (np.concatenate(rows_P), np.concatenate(cols_P))),
                      shape=(int(offs[-1]), int(coffs[-1])))
    return P, s_agg, svals


def blockdiag_csr(Binv):
    if isinstance(Binv, BlockDiag):
        return Binv.to_csr()
    nun, nb, _ = Binv.shape
    return sp.block_diag(list(Binv), format="csr") if nun < 64 else sp.bsr_matrix(
        (Binv, np.arange(nun), np.arange(nun + 1)), shape=(nun * nb, nun * nb)).tocsr()


def smoothed_prolongator(A, Dinv, omega, P):
    """eq:TR0: T = (I - omega D^{-1} A) P and R = T^T."""
    T = (P - omega * (blockdiag_csr(Dinv) @ (A @ P))).tocsr()
    return T, T.T.tocsr()


def galerkin(R, A, T):
    """A_{k+1} = R A_k T."""
    return (R @ (A @ T)).tocsr()


# --------------------------------------------------------------------------
# whole setup
# --------------------------------------------------------------------------

def setup(A0, nb, aggs, params, B1, b_update="R"):
    """Algorithm 5.  A0: scipy sparse (n x n); aggs: per-level unit->aggregate
    maps (from rcb.rcb_hierarchy; a map that is the identity replicates a level,
    the h*-step of Algorithm 5's intra-element coarsening); B1: n x r initial
    candidates.  params.delta (default 1e-3, Section 4.3) is the h*-threshold.

    Reading of the h*-step (a replicated level, every aggregate one unit): the
    text says it differs from an h-step only in its aggregates and s_J, which
    would smooth P~ as in eq:TR0; the paper's printed h*-hierarchy (level-1
    nonzeros equal to the elements' face stencil times s^2) fits T = P~ (no
    smoothing, R = P~^T) instead, whose coarse operator keeps the fine face
    stencil where the smoothed one spans three rings of neighbours.  The
    unsmoothed form is the default; params.hstar_smooth = True takes eq:TR0.

    b_update 'R' initialises B^{k+1} = R B^k (Algorithm 5); 'P' uses P^T B^k
    (eq:SA_Bk)."""
    N = len(aggs)
    A = A0.tocsr().astype(np.float64)
    nunits = A.shape[0] // nb
    sizes = np.full(nunits, nb, dtype=np.int64)
    delta = float(getattr(params, "delta", 1e-3))
    B = np.array(B1, dtype=np.float64, copy=True)
    if B.ndim == 1:
        B = B[:, None]
    levels = []
    for k in range(N):
        uniform = bool(np.all(sizes == sizes[0]))
        L = Level(A=A, nb=int(sizes[0]) if uniform else 0, nunits=nunits, sizes=sizes)
        L.Dinv_bd = BlockDiag.from_matrix(A, sizes).inverse()
        if uniform:
            L.Dinv = L.Dinv_bd.uniform_array()
        if params.omega_fixed > 0:
            L.omega = float(params.omega_fixed)
        else:
            x0 = uniform_pm1(params.pow_seed + k, A.shape[0])
            L.rho = power_rho(A, L.Dinv_bd, 0, params.q_power, x0)
            L.omega = omega_from_rho(L.rho)
        L.B_in = B.copy()
        cols, sw = [], []
        for j in range(B.shape[1]):
            xj, mj = relax_candidate(A, L.Dinv_bd, 0, L.omega, B[:, j].copy(), params.gamma, params.relax_max)
            cols.append(xj)
            sw.append(mj)
        L.B = np.stack(cols, axis=1)
        L.sweeps = np.array(sw)
        L.agg = np.asarray(aggs[k], dtype=np.int64)
        L.P, L.s_agg, L.sv = tentative_prolongator(L.B, L.agg, sizes, params.n_cut, delta)
        L.s = int(L.s_agg.max())
        replicated = len(np.unique(L.agg)) == nunits          # every aggregate is a single unit
        if replicated and not getattr(params, "hstar_smooth", False):
            L.T, L.R = L.P.tocsr(), L.P.T.tocsr()              # unsmoothed h*-step (see setup's docstring)
        else:
            L.T, L.R = smoothed_prolongator(A, L.Dinv_bd, L.omega, L.P)
        Anext = galerkin(L.R, A, L.T)
        B = (L.R @ L.B) if b_update == "R" else (L.P.T @ L.B)
        levels.append(L)
        A, sizes, nunits = Anext, L.s_agg.copy(), int(L.agg.max()) + 1
    uniform = bool(np.all(sizes == sizes[0]))
    levels.append(Level(A=A, nb=int(sizes[0]) if uniform else 0, nunits=nunits, sizes=sizes))
    lu = sla.lu_factor(A.toarray())
    return Hierarchy(levels, lu, params.t_pre, params.t_post)


# --------------------------------------------------------------------------
# V-cycle (Algorithms 1 and 2)
# --------------------------------------------------------------------------

def smooth(A, Dinv, nb, omega, b, u, sweeps):
    """Algorithm 1 with the block Jacobi smoother A~ = D / omega (eq:smoother_choice):
    u <- u + omega D^{-1} (b - A u), a fixed number of sweeps."""
    for _ in range(sweeps):
        u = u + omega * _apply_dinv(Dinv, b - A @ u, nb)
    return u


def vcycle(H, b):
    """One V-cycle for A u = b from u = 0 (Algorithm 2, one pass).

    Down: u_k = Smooth(0, ..., t_pre); r_k = b_k - A_k u_k; b_{k+1} = R r_k.
    Bottom: u_N = A_N^{-1} b_N.  Up: u_k += T u_{k+1}, then t_post sweeps on
    A_k u = b_k.  Reading: the post-smoothing right-hand side of the listing is
    taken as b_k (the standard V-cycle)."""
    Ls = H.levels
    N = len(Ls) - 1
    bs, us = [None] * (N + 1), [None] * (N + 1)
    bs[0] = b
    for k in range(N):
        L = Ls[k]
        u = L.omega * L.Dinv_bd.apply(bs[k])                          # first sweep from zero
        u = smooth(L.A, L.Dinv_bd, 0, L.omega, bs[k], u, H.t_pre - 1)
        us[k] = u
        bs[k + 1] = L.R @ (bs[k] - L.A @ u)
    us[N] = sla.lu_solve(H.lu, bs[N])
    for k in range(N - 1, -1, -1):
        L = Ls[k]
        u = us[k] + L.T @ us[k + 1]
        us[k] = smooth(L.A, L.Dinv_bd, 0, L.omega, bs[k], u, H.t_post)
    return us[0]


def to_fp32(H):
    """FP32 copies of every level operator (rounded to nearest), the coarsest LU
    kept in FP64 (mixed-precision V-cycle)."""
    L32 = []
    for L in H.levels[:-1]:
        L32.append(dict(A=L.A.astype(np.float32), Dinv=L.Dinv_bd.astype(np.float32),
                        omega=np.float32(L.omega), T=L.T.astype(np.float32), R=L.R.astype(np.float32)))
    return L32


def vcycle_fp32(H, L32, b):
    """The V-cycle of ``vcycle`` computed in FP32 (FP32 operators, FP32 vector
    arithmetic) except the coarsest solve, done in FP64 on the rounded-up b_N."""
    N = len(L32)
    bs, us = [None] * (N + 1), [None] * (N + 1)
    bs[0] = np.asarray(b, dtype=np.float32)
    for k in range(N):
        L = L32[k]
        u = L["omega"] * L["Dinv"].apply(bs[k])
        for _ in range(H.t_pre - 1):
            u = u + L["omega"] * L["Dinv"].apply(bs[k] - L["A"] @ u)
        us[k] = u
        bs[k + 1] = (L["R"] @ (bs[k] - L["A"] @ u)).astype(np.float32)
    us[N] = sla.lu_solve(H.lu, bs[N].astype(np.float64)).astype(np.float32)
    for k in range(N - 1, -1, -1):
        L = L32[k]
        u = us[k] + L["T"] @ us[k + 1]
        for _ in range(H.t_post):
            u = u + L["omega"] * L["Dinv"].apply(bs[k] - L["A"] @ u)
        us[k] = u
    return us[0].astype(np.float32)


# --------------------------------------------------------------------------
# block patterns (structural, for index parity)
# --------------------------------------------------------------------------

def block_patterns(A0_row_ptr, A0_col_idx, aggs, hstar_smooth=False):
    """Structural block patterns per level: T (unit x aggregate), A_{k+1}.

    T block (e, J) exists iff J is e's aggregate or the aggregate of a block
    column of row e of A_k (eq:TR0, no numerical dropping); on a replicated
    level (every aggregate one unit) T = P~ holds e's own aggregate only
    unless hstar_smooth.  A_{k+1} block (I, J) exists iff T(a, I), A_k(a, b)
    and T(b, J) all exist."""
    n0 = len(A0_row_ptr) - 1
    Apat = sp.csr_matrix((np.ones(len(A0_col_idx), dtype=np.int64), A0_col_idx, A0_row_ptr), shape=(n0, n0))
    out = []
    for agg in aggs:
        nun = Apat.shape[0]
        nag = int(agg.max()) + 1
        G = sp.csr_matrix((np.ones(nun, dtype=np.int64), (np.arange(nun), agg)), shape=(nun, nag))
        Tpat = G.tocsr() if (nag == nun and not hstar_smooth) else (G + Apat @ G).tocsr()
        Tpat.data[:] = 1
        Tpat.sort_indices()
        Anext = (Tpat.T @ Apat @ Tpat).tocsr()
        Anext.data[:] = 1
        Anext.sort_indices()
        out.append(dict(T_ptr=Tpat.indptr.astype(np.int32), T_idx=Tpat.indices.astype(np.int32),
                        A_ptr=Anext.indptr.astype(np.int32), A_idx=Anext.indices.astype(np.int32)))
        Apat = Anext
    return out
