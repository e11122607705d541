"""DG discretisations of Poisson's problem on the structured hexahedral mesh of
Section 5.1 (input generation only).

Domain [-1, 1]^3 cut into 2^M cubes per direction (h = 2 / 2^M), outer-product
polynomials of degree p in every element (Q_p, nb = (p+1)^3), homogeneous
Dirichlet data on the face x = -1 and Neumann data on the five other faces.
The paper's manufactured solution vanishes on x = -1, so homogeneous Dirichlet
data is all that problem needs; only that case is supported here.

Basis: on each element the products psi_a(tx) psi_b(ty) psi_c(tz) of the
Legendre polynomials orthonormal on [0, 1] (t the element-local coordinate),
local index (a (p+1) + b)(p+1) + c; the element mass matrix is h^3 I, as for
the simplex workloads.  Elements are numbered (ix n1 + iy) n1 + iz, n1 = 2^M.

Because the mesh is uniform and the basis a tensor product, each of the three
directional parts of either bilinear form is a one-dimensional DG operator
along that direction times the (diagonal, h I) mass matrices along the other
two.  The operator is assembled as that sum of three Kronecker products and
permuted into element-block (BSR) order.

* IP (symmetric interior penalty): volume term, the consistency and symmetry
  terms on interior and Dirichlet faces, and the penalty mu / h on the jumps
  there, mu = M (p+1)^2 / 2 (Section 5.1; the reading that mu multiplies 1/h
  is this module's).
* LDG, minimal dissipation: the lifted gradient takes the trace from the
  element on the lower-coordinate side of every interior face (one consistent
  switch direction, (1, 1, 1)) and zero on the Dirichlet face; no interior
  penalty; the Dirichlet face carries the penalty mu / h.  The primal form is
  sum_K (q(u), q(v))_K + Dirichlet penalty, and on this mesh its block pattern
  is the seven-point face stencil, like IP.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg

from . import dg


def penalty_mu(M, p):
    """IP penalty parameter of Section 5.1: M (p+1)^2 / 2."""
    return M * (p + 1) ** 2 / 2.0


@dataclass
class HexMesh:
    """Uniform Cartesian mesh of [-1, 1]^3 with 2^M cubes per direction."""
    M: int
    dim: int = 3

    @property
    def n1(self):
        return 2 ** self.M

    @property
    def h(self):
        return 2.0 / self.n1

    @property
    def n_elem(self):
        return self.n1 ** 3

    def index(self):
        """(ix, iy, iz) of every element, in element order."""
        i = np.arange(self.n_elem)
        n1 = self.n1
        return i // (n1 * n1), (i // n1) % n1, i % n1

    def centroids(self):
        ix, iy, iz = self.index()
        return np.stack([-1.0 + (ix + 0.5) * self.h, -1.0 + (iy + 0.5) * self.h,
                         -1.0 + (iz + 0.5) * self.h], axis=1)

    def adjacency(self):
        """Face-neighbour graph as CSR (int32 ptr, int32 idx), columns sorted."""
        n1 = self.n1
        ix, iy, iz = self.index()
        e = np.arange(self.n_elem)
        rows, cols = [], []
        for d, (c, stride) in enumerate(((ix, n1 * n1), (iy, n1), (iz, 1))):
            for step in (-1, 1):
                ok = (c + step >= 0) & (c + step < n1)
                rows.append(e[ok])
                cols.append(e[ok] + step * stride)
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        order = np.lexsort((c, r))
        r, c = r[order], c[order]
        ptr = np.zeros(self.n_elem + 1, dtype=np.int64)
        np.add.at(ptr, r + 1, 1)
        return np.cumsum(ptr).astype(np.int32), c.astype(np.int32)


# ----------------------------------------------------------------------------
# one-dimensional building blocks
# ----------------------------------------------------------------------------

def _psi(p, t):
    """Legendre polynomials orthonormal on [0, 1] and their t-derivatives at t: (len(t), p+1) each."""
    t = np.asarray(t, dtype=np.float64)
    val = np.empty(t.shape + (p + 1,))
    der = np.empty(t.shape + (p + 1,))
    for i in range(p + 1):
        c = np.zeros(i + 1)
        c[i] = np.sqrt(2 * i + 1)
        val[..., i] = npleg.legval(2 * t - 1, c)
        der[..., i] = 2 * npleg.legval(2 * t - 1, npleg.legder(c))
    return val, der


def _gauss01(n):
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


class _Line:
    """One-dimensional element quantities for element size h."""

    def __init__(self, p, h):
        self.p, self.h, self.k = p, h, p + 1
        tq, wq = _gauss01(p + 1)
        val, der = _psi(p, tq)
        self.K = (der * wq[:, None]).T @ der / h           # int phi_i' phi_j' dx
        self.C = (val * wq[:, None]).T @ der                # C[i, j] = int psi_i psi_j' dt
        (v0, v1), (d0, d1) = _psi(p, np.array([0.0, 1.0]))
        self.v0, self.v1 = v0, v1                           # traces at the element's ends
        self.d0, self.d1 = d0 / h, d1 / h                   # x-derivatives there


def _blocks_to_csr(n_el, k, blocks):
    """Assemble {(row elem, col elem): dense k x k block} into a CSR matrix of size n_el k."""
    R, C, D = [], [], []
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    for (a, b), blk in blocks.items():
        R.append(a * k + ii.ravel())
        C.append(b * k + jj.ravel())
        D.append(np.asarray(blk).ravel())
    n = n_el * k
    return sp.csr_matrix((np.concatenate(D), (np.concatenate(R), np.concatenate(C))), shape=(n, n))


def _add(blocks, key, blk):
    blocks[key] = blocks[key] + blk if key in blocks else blk.copy()


def ip_1d(n1, p, h, sigma, dirichlet_left, dirichlet_right):
    """IP operator along one direction: volume, interior points (normal +x
    from the left element P to the right element M) and Dirichlet ends."""
    L = _Line(p, h)
    blocks = {}
    for e in range(n1):
        _add(blocks, (e, e), L.K)
    # side data at an interior point: (trace, normal derivative, sign of the jump)
    side = {0: (L.v1, L.d1, 1.0), 1: (L.v0, L.d0, -1.0)}
    for e in range(n1 - 1):
        for s in (0, 1):
            vs, ds, cs = side[s]
            for t in (0, 1):
                vt, dt, ct = side[t]
                blk = (-0.5 * cs * np.outer(vs, dt) - 0.5 * ct * np.outer(ds, vt)
                       + cs * ct * sigma * np.outer(vs, vt))
                _add(blocks, (e + s, e + t), blk)
    ends = []
    if dirichlet_left:
        ends.append((0, L.v0, -L.d0))
    if dirichlet_right:
        ends.append((n1 - 1, L.v1, L.d1))
    for e, v, dn in ends:
        _add(blocks, (e, e), -np.outer(v, dn) - np.outer(dn, v) + sigma * np.outer(v, v))
    return _blocks_to_csr(n1, L.k, blocks)


def ldg_1d(n1, p, h, sigma, dirichlet_left, dirichlet_right):
    """LDG (minimal dissipation) operator along one direction: D^T (h I) D plus
    the penalty at Dirichlet ends, D the lifted derivative with the trace taken
    from the left element at interior points, zero at Dirichlet ends and the
    element's own at Neumann ends."""
    L = _Line(p, h)
    g = {}
    for e in range(n1):
        _add(g, (e, e), L.C)
    # left end of element e+1 (outward normal -1): -(u_e(1) - u_{e+1}(0)) psi(0)
    for e in range(n1 - 1):
        _add(g, (e + 1, e), -np.outer(L.v0, L.v1))
        _add(g, (e + 1, e + 1), np.outer(L.v0, L.v0))
    if dirichlet_left:
        _add(g, (0, 0), np.outer(L.v0, L.v0))
    if dirichlet_right:
        _add(g, (n1 - 1, n1 - 1), -np.outer(L.v1, L.v1))
    D = _blocks_to_csr(n1, L.k, g) / h          # mass h I on the lifted side
    A = (D.T @ D) * h
    pen = {}
    if dirichlet_left:
        _add(pen, (0, 0), sigma * np.outer(L.v0, L.v0))
    if dirichlet_right:
        _add(pen, (n1 - 1, n1 - 1), sigma * np.outer(L.v1, L.v1))
    if pen:
        A = A + _blocks_to_csr(n1, L.k, pen)
    return A.tocsr()


# ----------------------------------------------------------------------------
# three-dimensional operator
# ----------------------------------------------------------------------------

def _tensor_to_block_perm(n1, k):
    """perm[i] = tensor-order index of block-order dof i."""
    e = np.arange(n1 ** 3)
    ix, iy, iz = e // (n1 * n1), (e // n1) % n1, e % n1
    a, b, c = np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    N = n1 * k
    X = ix[:, None] * k + a[None, :]
    Y = iy[:, None] * k + b[None, :]
    Z = iz[:, None] * k + c[None, :]
    return ((X * N + Y) * N + Z).ravel()


def assemble_hex(M, p, flux="ip"):
    """Poisson operator on the 2^M-per-direction hex mesh, Q_p, flux 'ip' or
    'ldg'; Dirichlet on x = -1, Neumann elsewhere.  Returns a dg.BSR."""
    mesh = HexMesh(M)
    n1, h, k = mesh.n1, mesh.h, p + 1
    sigma = penalty_mu(M, p) / h
    one_d = {"ip": ip_1d, "ldg": ldg_1d}[flux]
    Ax = one_d(n1, p, h, sigma, True, False)
    An = one_d(n1, p, h, sigma, False, False)
    Mm = sp.identity(n1 * k, format="csr") * h
    A = (sp.kron(Ax, sp.kron(Mm, Mm)) + sp.kron(Mm, sp.kron(An, Mm))
         + sp.kron(Mm, sp.kron(Mm, An))).tocsr()
    perm = _tensor_to_block_perm(n1, k)
    A = A[perm][:, perm]
    return dg.csr_to_bsr(A, k ** 3, mesh.n_elem)


# ----------------------------------------------------------------------------
# right-hand sides
# ----------------------------------------------------------------------------

def _elem_origin(mesh):
    ix, iy, iz = mesh.index()
    return np.stack([ix, iy, iz], axis=1) * mesh.h - 1.0


def load_vector(M, p, f, grad_u, nq=None, chunk=4096):
    """b_i = int f phi_i + int_{Neumann faces} (grad u . n) phi_i for callables
    f(x) and grad_u(x) on (N, 3) points; homogeneous Dirichlet data on x = -1."""
    mesh = HexMesh(M)
    h, k = mesh.h, p + 1
    nq = nq or p + 4
    tq, wq = _gauss01(nq)
    psi, _ = _psi(p, tq)                                  # (q, k)
    org = _elem_origin(mesh)
    b = _volume(M, p, f, nq, chunk).reshape(-1, k, k, k)
    # Neumann faces: every boundary face except x = -1
    T2 = np.stack(np.meshgrid(tq, tq, indexing="ij"), axis=-1).reshape(-1, 2)
    W2 = wq[:, None] * wq[None, :]
    ends = _psi(p, np.array([0.0, 1.0]))[0]              # (2, k): traces at t = 0, 1
    ix, iy, iz = mesh.index()
    coord = (ix, iy, iz)
    for ax in range(3):
        others = [d for d in range(3) if d != ax]
        for side in (0, 1):
            if ax == 0 and side == 0:
                continue
            sel = np.nonzero(coord[ax] == (0 if side == 0 else mesh.n1 - 1))[0]
            x = np.repeat(org[sel][:, None, :], len(T2), axis=1)
            x[:, :, ax] = -1.0 if side == 0 else 1.0
            x[:, :, others[0]] += h * T2[None, :, 0]
            x[:, :, others[1]] += h * T2[None, :, 1]
            n = np.zeros(3)
            n[ax] = -1.0 if side == 0 else 1.0
            g = (grad_u(x.reshape(-1, 3)) @ n).reshape(len(sel), nq, nq) * W2
            face = h ** 2 * np.einsum("euv,ua,vb->eab", g, psi, psi, optimize=True)
            tr = ends[side]
            if ax == 0:
                b[sel] += tr[None, :, None, None] * face[:, None, :, :]
            elif ax == 1:
                b[sel] += tr[None, None, :, None] * face[:, :, None, :]
            else:
                b[sel] += tr[None, None, None, :] * face[:, :, :, None]
    return b.reshape(-1)


def project(M, p, u, nq=None):
    """Coefficients of the L2 projection of u onto the Q_p space (mass h^3 I)."""
    return _volume(M, p, u, nq) / HexMesh(M).h ** 3


def _volume(M, p, f, nq=None, chunk=4096):
    """int_K f phi_i for every element K and local function i (tensor Gauss
    rule with nq points per direction), flattened in element-block order."""
    mesh = HexMesh(M)
    h, k, ne = mesh.h, p + 1, mesh.n_elem
    nq = nq or p + 4
    tq, wq = _gauss01(nq)
    psi, _ = _psi(p, tq)
    org = _elem_origin(mesh)
    T = np.stack(np.meshgrid(tq, tq, tq, indexing="ij"), axis=-1).reshape(-1, 3)
    W = (wq[:, None, None] * wq[None, :, None] * wq[None, None, :])
    out = np.zeros((ne, k, k, k))
    for s in range(0, ne, chunk):
        o = org[s:s + chunk]
        x = o[:, None, :] + h * T[None, :, :]
        fx = f(x.reshape(-1, 3)).reshape(len(o), nq, nq, nq) * W
        out[s:s + chunk] = h ** 3 * np.einsum("exyz,xa,yb,zc->eabc", fx, psi, psi, psi, optimize=True)
    return out.reshape(-1)


# ----------------------------------------------------------------------------
# the manufactured solution of Section 5.1: u = exp(sin(pi x) sin(pi y) sin(pi z)) - 1
# ----------------------------------------------------------------------------

def _s_and_grad(x):
    sx, sy, sz = (np.sin(np.pi * x[:, d]) for d in range(3))
    cx, cy, cz = (np.cos(np.pi * x[:, d]) for d in range(3))
    s = sx * sy * sz
    gs = np.pi * np.stack([cx * sy * sz, sx * cy * sz, sx * sy * cz], axis=1)
    return s, gs


def paper_u(x):
    s, _ = _s_and_grad(x)
    return np.exp(s) - 1.0


def paper_grad_u(x):
    s, gs = _s_and_grad(x)
    return np.exp(s)[:, None] * gs


def paper_f(x):
    """-Laplace(u) = exp(s) (3 pi^2 s - |grad s|^2)."""
    s, gs = _s_and_grad(x)
    return np.exp(s) * (3.0 * np.pi ** 2 * s - (gs ** 2).sum(axis=1))


def paper_rhs(M, p):
    """Load vector of the manufactured solution: volume term and Neumann data."""
    return load_vector(M, p, paper_f, paper_grad_u)
