"""Seeded synthetic workloads (input generation only; no multigrid arithmetic).

Each workload bundles a mesh, its DG matrix in BSR form, right-hand side(s),
the initial adaptive candidates B^1 and the method parameters.  Seeds: mesh 0,
right-hand side 1, B^1 2.  Sizes follow the benchmark configurations:

* ``poisson2d_p1_16``  : 16x16 split squares, SIPG p=1 (512 triangles, 1,536 dofs)
* ``poisson2d_p3_256`` : Delaunay of 256^2 jittered points, SIPG p=3
                         (130,050 triangles, 1,300,500 dofs)
* ``convdiff2d_p2_363``: Delaunay of 363^2 jittered points, LDG + upwind p=2
                         (262,088 triangles, 1,572,528 dofs)
* ``poisson3d_p2_64``  : 64^3 jittered Kuhn cube, SIPG p=2
                         (1,572,864 tetrahedra, 15,728,640 dofs)

* ``poisson3d_hex``    : the structured test problem of Section 5.1: 2^M hexahedra
                         per direction on [-1, 1]^3, Q1 (nb = 8), IP or LDG,
                         Dirichlet on x = -1, Neumann elsewhere, right-hand
                         side of the paper's manufactured solution
                         (M = 4: 4,096 hexahedra, 32,768 dofs)

* ``serving_catalogue``: the operator instances of the serving stream (2D
                         jittered Delaunay meshes of 1k-200k triangles, p = 1..4,
                         SIPG-Poisson or LDG + upwind convection-diffusion)

Scaled-down variants (same recipe, fewer elements) are used by the tests.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import dg, hexdg, mesh as meshes


@dataclass
class Params:
    n_levels: int                 # levels L_0..L_{n_levels-1}
    bisections: int               # binary splits per level (2^b-way aggregation)
    r: int                        # adaptive candidates
    t_pre: int = 3
    t_post: int = 3
    omega_fixed: float = 0.0      # 0 -> adaptive omega from the power iteration
    gamma: float = 0.03
    q_power: int = 3
    relax_max: int = 100
    n_cut: float = 3.0
    pow_seed: int = 3
    delta: float = 1e-3           # h*-step threshold of eq:sik (Section 4.3)
    hstar_top: bool = False       # replicate level 0 (an h*-step before the geometric levels)
    hstar_smooth: bool = False    # smooth P~ on the replicated level too (eq:TR0) instead of T = P~


@dataclass
class Workload:
    name: str
    mesh: object
    p: int
    A: dg.BSR
    b: np.ndarray
    B1: np.ndarray
    params: Params
    krylov: str                   # "pcg" | "gmres"
    tol: float = 1e-8
    extra: dict = field(default_factory=dict)

    @property
    def centroids(self):
        return np.ascontiguousarray(self.mesh.centroids())

    @property
    def adjacency(self):
        return self.mesh.adjacency()


def n_cut_default(dim):
    """n_cut = 2^d - (d - 1) (Section 4.3)."""
    return float(2 ** dim - (dim - 1))


def _finish(name, m, p, A, params, krylov, rhs_kind="normal", n_rhs=1, extra=None):
    n = A.n
    rng_b = np.random.default_rng(1)
    if rhs_kind == "normal":
        b = rng_b.standard_normal((n, n_rhs))
    else:
        b = rng_b.uniform(-1.0, 1.0, (n, n_rhs))
    if n_rhs == 1:
        b = b[:, 0]
    B1 = np.random.default_rng(2).standard_normal((n, params.r))
    return Workload(name, m, p, A, np.ascontiguousarray(b), np.ascontiguousarray(B1), params, krylov,
                    extra=extra or {})


def poisson2d_split(nx=16, p=1, n_levels=3, bisections=3, r=1, nu=1, omega=0.7, n_rhs=1):
    m = meshes.split_square(nx)
    A = dg.assemble_sipg(m, p)
    prm = Params(n_levels, bisections, r, nu, nu, omega_fixed=omega, n_cut=n_cut_default(2))
    return _finish(f"poisson2d_p{p}_split{nx}", m, p, A, prm, "pcg", n_rhs=n_rhs)


def poisson2d_delaunay(side=256, p=3, n_levels=5, bisections=2, r=3, nu=3, n_rhs=1):
    m = meshes.jittered_delaunay(side, 0.25, seed=0)
    A = dg.assemble_sipg(m, p)
    prm = Params(n_levels, bisections, r, nu, nu, n_cut=n_cut_default(2))
    return _finish(f"poisson2d_p{p}_delaunay{side}", m, p, A, prm, "pcg", n_rhs=n_rhs)


def convdiff2d_delaunay(side=363, p=2, peclet=1e2, n_levels=6, bisections=2, r=4, nu=3, n_rhs=1):
    m = meshes.jittered_delaunay(side, 0.25, seed=0)
    beta = np.array([np.cos(0.3), np.sin(0.3)])
    A = dg.assemble_ldg_upwind(m, p, beta, 1.0 / peclet)
    prm = Params(n_levels, bisections, r, nu, nu, n_cut=n_cut_default(2))
    return _finish(f"convdiff2d_p{p}_delaunay{side}_pe{peclet:g}", m, p, A, prm, "gmres",
                   rhs_kind="uniform", n_rhs=n_rhs, extra={"peclet": peclet})


def poisson3d_kuhn(n=64, p=2, n_levels=5, bisections=3, r=4, nu=2, n_rhs=1, log=None):
    m = meshes.kuhn_cube(n, 0.2, seed=0)
    A = dg.assemble_sipg(m, p, log=log)
    prm = Params(n_levels, bisections, r, nu, nu, n_cut=n_cut_default(3))
    return _finish(f"poisson3d_p{p}_kuhn{n}", m, p, A, prm, "pcg", n_rhs=n_rhs)


def poisson3d_hex(M=4, p=1, flux="ip", r=8, nu=3, n_levels=None, rhs="paper", relax_max=100, hstar=False):
    """Section 5.1's structured Poisson problem.  Levels: ceil(log_8 |T_h|), so
    that the coarsest level holds 8 aggregates, with 8-way aggregation per
    level; with hstar, level 0 is replicated first (the h*-step of Section 4.3,
    one more level).  rhs "paper" is the load vector of the manufactured
    solution, else seeded N(0, 1) like the other workloads."""
    m = hexdg.HexMesh(M)
    A = hexdg.assemble_hex(M, p, flux)
    if n_levels is None:
        n_levels = max(2, M) + (1 if hstar else 0)
    prm = Params(n_levels, 3, r, nu, nu, relax_max=relax_max, n_cut=n_cut_default(3), hstar_top=hstar)
    w = _finish(f"poisson3d_hex{M}_q{p}_{flux}{'_hstar' if hstar else ''}", m, p, A, prm, "pcg",
                extra={"flux": flux, "M": M})
    if rhs == "paper":
        w.b = np.ascontiguousarray(hexdg.paper_rhs(M, p))
        w.tol = 1e-7
    return w


def levels_for_coarsest(n_elem, bisections=2, r=3, max_coarse=2048):
    """Fewest levels whose coarsest level has at most max_coarse dofs: level k
    holds 2^(D - k*bisections) aggregates (D = ceil(log2 n_elem)) of r dofs."""
    D = max(1, math.ceil(math.log2(max(n_elem, 2))))
    N = 1
    while D - N * bisections > 0 and (2 ** (D - N * bisections)) * r > max_coarse:
        N += 1
    return N + 1


def serving_catalogue(n_ops=32, t_min=1e3, t_max=2e5, seed=0, log=None):
    """Operator instances of the serving stream.  Per instance i (parameters
    from one generator seeded `seed`): triangle count T log-uniform in
    [t_min, t_max] (grid side round(sqrt(T/2)) + 1, mesh seed i), p uniform in
    {1, 2, 3, 4}, and with probability 1/2 each SIPG-Poisson (PCG, N(0,1)
    right-hand sides) or LDG + upwind convection-diffusion with Peclet number
    log-uniform in [1, 1e4] (FGMRES, U(-1, 1) right-hand sides).  r = 3,
    V(3,3), levels chosen so that the coarsest level has at most 2,048 dofs.
    Aggregation is 4-way per level for p >= 2 and 8-way for p = 1 (as in the
    16x16 p=1 workload): a level-1 aggregate then holds at least 12 dofs, so
    every aggregate keeps s = r = 3 coarse dofs."""
    rng = np.random.default_rng(seed)
    out = []
    beta = np.array([np.cos(0.3), np.sin(0.3)])
    for i in range(n_ops):
        T = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
        side = int(round(math.sqrt(T / 2.0))) + 1
        p = int(rng.integers(1, 5))
        sipg = bool(rng.random() < 0.5)
        pe = float(10.0 ** rng.uniform(0.0, 4.0))
        m = meshes.jittered_delaunay(side, 0.25, seed=i)
        bis = 3 if p == 1 else 2
        prm = Params(levels_for_coarsest(m.n_elem, bis), bis, 3, 3, 3, n_cut=n_cut_default(2))
        if sipg:
            A = dg.assemble_sipg(m, p)
            w = _finish(f"serve{i}_sipg_p{p}_{m.n_elem}", m, p, A, prm, "pcg")
        else:
            A = dg.assemble_ldg_upwind(m, p, beta, 1.0 / pe)
            w = _finish(f"serve{i}_ldg_p{p}_{m.n_elem}_pe{pe:.3g}", m, p, A, prm, "gmres", rhs_kind="uniform",
                        extra={"peclet": pe})
        if log:
            log(f"catalogue {i}: {w.name}, {A.n} dofs, {prm.n_levels} levels")
        out.append(w)
    return out
