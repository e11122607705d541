"""Checks of the structured hexahedral input generator (Section 5.1's test
problem: Q_p on 2^M cubes per direction of [-1, 1]^3, Dirichlet on x = -1,
Neumann elsewhere), for both fluxes (IP and minimal-dissipation LDG).

* Polynomial exactness: both discretisations are consistent, so for a
  solution in Q_p that vanishes on x = -1 the discrete solution is its L2
  projection up to rounding.  This exercises every volume, interior-face,
  Dirichlet-face and Neumann-face term and the load vector.
* Convergence at order p+1 for the paper's manufactured solution.
* Symmetry, definiteness, the seven-point block pattern and the level count
  of the paper (coarsest level: 2^d aggregates).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import amg, krylov, rcb
from workloads import configs, hexdg


def _poly(p):
    """(u, grad u, f = -Laplace u) for a Q_p polynomial with u = 0 on x = -1."""
    if p == 1:
        u = lambda x: (x[:, 0] + 1) * (1 + x[:, 1]) * x[:, 2]  # noqa: E731
        g = lambda x: np.stack([(1 + x[:, 1]) * x[:, 2], (x[:, 0] + 1) * x[:, 2],  # noqa: E731
                                (x[:, 0] + 1) * (1 + x[:, 1])], 1)
        f = lambda x: np.zeros(len(x))  # noqa: E731
        return u, g, f

    def u(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return (X + 1) * (X * Y ** 2 - Z + 0.5 * Y * Z)

    def g(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return np.stack([2 * X * Y ** 2 + Y ** 2 - Z + 0.5 * Y * Z,
                         2 * X ** 2 * Y + 2 * X * Y + 0.5 * (X * Z + Z),
                         -X - 1 + 0.5 * (X * Y + Y)], 1)

    def f(x):
        X, Y = x[:, 0], x[:, 1]
        return -(2 * Y ** 2 + 2 * X ** 2 + 2 * X)

    return u, g, f


@pytest.mark.parametrize("flux", ["ip", "ldg"])
@pytest.mark.parametrize("p", [1, 2])
def test_polynomial_exactness(flux, p):
    u, g, f = _poly(p)
    M = 2
    A = hexdg.assemble_hex(M, p, flux).to_scipy().tocsc()
    c = spla.spsolve(A, hexdg.load_vector(M, p, f, g))
    cp = hexdg.project(M, p, u)
    assert np.abs(cp).max() > 0.1
    assert np.abs(c - cp).max() <= 1e-11 * np.abs(cp).max()


@pytest.mark.parametrize("flux", ["ip", "ldg"])
def test_paper_solution_converges_at_order_p_plus_1(flux):
    p, errs = 2, []
    for M in (2, 3):
        A = hexdg.assemble_hex(M, p, flux).to_scipy().tocsc()
        c = spla.spsolve(A, hexdg.paper_rhs(M, p))
        cp = hexdg.project(M, p, hexdg.paper_u)
        errs.append(np.sqrt(hexdg.HexMesh(M).h ** 3 * ((c - cp) ** 2).sum()))
    assert errs[1] < 0.01
    assert np.log2(errs[0] / errs[1]) > 2.5


@pytest.mark.parametrize("flux", ["ip", "ldg"])
def test_structure(flux):
    M, p = 2, 1
    mesh = hexdg.HexMesh(M)
    B = hexdg.assemble_hex(M, p, flux)
    n1 = mesh.n1
    assert B.nb == (p + 1) ** 3 and B.n_brow == n1 ** 3
    assert B.nnzb == n1 ** 3 + 6 * n1 * n1 * (n1 - 1)
    ptr, idx = mesh.adjacency()
    for e in range(mesh.n_elem):
        cols = set(B.col_idx[B.row_ptr[e]:B.row_ptr[e + 1]].tolist())
        assert cols == set(idx[ptr[e]:ptr[e + 1]].tolist()) | {e}
    A = B.to_scipy().toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)


def test_neighbours_and_centroids():
    mesh = hexdg.HexMesh(3)
    c = mesh.centroids()
    ptr, idx = mesh.adjacency()
    e = np.repeat(np.arange(mesh.n_elem), np.diff(ptr))
    d = np.abs(c[e] - c[idx]).sum(1)
    assert np.allclose(d, mesh.h)
    assert np.diff(ptr).min() == 3 and np.diff(ptr).max() == 6


def test_levels_end_at_2_to_the_d_aggregates():
    w = configs.poisson3d_hex(3)
    aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
    assert w.params.n_levels == 3 and len(np.unique(aggs[-1])) == 8


@pytest.mark.parametrize("flux", ["ip", "ldg"])
def test_oracle_multigrid_converges_on_hex(flux):
    w = configs.poisson3d_hex(3, flux=flux)
    A = w.A.to_scipy()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
    H = amg.setup(A, w.A.nb, aggs, w.params, w.B1)
    x, it, _ = krylov.pcg(A, w.b, lambda r: amg.vcycle(H, r), 1e-7, 100)[:3]
    assert it <= 20
    assert np.linalg.norm(w.b - A @ x) <= 1e-7 * np.linalg.norm(w.b)
