"""DG discretisations on simplex meshes, assembled into block-sparse (BSR) form.

Input generation only: this module produces the linear systems ``A u = f``
(Section 2, eq:ibp and eq:Auf) that the multigrid method consumes.  One dense
``nb x nb`` block is stored per element (diagonal) and per coupled element pair;
block row ``e`` holds the test functions of element ``e``.

* SIPG (symmetric interior penalty) for ``-Laplace(u) = f`` with homogeneous
  Dirichlet data imposed weakly on the whole boundary.  Penalty
  ``sigma_F = c p^2 / h_F`` with ``h_F = min(|K+|, |K-|) / |F|`` (boundary:
  ``|K| / |F|``).
* LDG with a switch along the convection direction (minimal dissipation:
  penalty on boundary faces only) plus upwind convection for
  ``-eps Laplace(u) + beta . grad(u) = f``.  LDG couples an element to the
  neighbours of its neighbours, so its block pattern is wider than the face
  graph.
"""
import numpy as np

from .basis import SimplexBasis
from .quadrature import gauss_line, gauss_tet, gauss_triangle


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _face_local_vertices(dim):
    return [[v for v in range(dim + 1) if v != f] for f in range(dim + 1)]


def _face_geometry(mesh, elem, lface):
    """Face vertices, outward unit normal (w.r.t. elem) and measure."""
    loc = np.array(_face_local_vertices(mesh.dim))
    fv = mesh.verts[np.take_along_axis(mesh.elems[elem], loc[lface], axis=1)]  # (nf, d, d)
    opp = mesh.verts[mesh.elems[elem, lface]]
    if mesh.dim == 2:
        t = fv[:, 1] - fv[:, 0]
        n = np.stack([t[:, 1], -t[:, 0]], axis=1)
        meas = np.linalg.norm(t, axis=1)
    else:
        n = np.cross(fv[:, 1] - fv[:, 0], fv[:, 2] - fv[:, 0])
        meas = 0.5 * np.linalg.norm(n, axis=1)
    n = n / np.linalg.norm(n, axis=1)[:, None]
    flip = np.einsum("fd,fd->f", n, fv[:, 0] - opp) < 0
    n[flip] *= -1.0
    return fv, n, meas


def _face_points(fv, dim, nq):
    """Physical quadrature points (nf, q, d) and weights (nf, q) on faces fv."""
    if dim == 2:
        t, w = gauss_line(nq)
        x = fv[:, None, 0] + t[None, :, None] * (fv[:, None, 1] - fv[:, None, 0])
        meas = np.linalg.norm(fv[:, 1] - fv[:, 0], axis=1)
        return x, w[None, :] * meas[:, None]
    xi, w = gauss_triangle(nq)
    a, b, c = fv[:, 0], fv[:, 1], fv[:, 2]
    x = a[:, None] + xi[None, :, 0, None] * (b - a)[:, None] + xi[None, :, 1, None] * (c - a)[:, None]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return x, 2.0 * w[None, :] * area[:, None]


def _wgram(w, a, b):
    """sum_q w[f,q] a[f,q,i] b[f,q,j] -> (f, i, j), as one batched product."""
    return np.matmul(np.swapaxes(a * w[..., None], -1, -2), b)


class _Geo:
    def __init__(self, mesh):
        self.J = mesh.jacobians()
        self.detJ = np.linalg.det(self.J)
        self.Jinv = np.linalg.inv(self.J)
        self.v0 = mesh.verts[mesh.elems[:, 0]]
        self.vol = np.abs(self.detJ) / (2.0 if mesh.dim == 2 else 6.0)

    def to_ref(self, elem, x):
        """Reference coordinates of physical points x (nf, q, d) in elements elem (nf,)."""
        return np.matmul(x - self.v0[elem][:, None, :], np.swapaxes(self.Jinv[elem], 1, 2))

    def phys_grad(self, elem, ghat):
        """Physical gradients from reference gradients ghat (nf, q, nb, d)."""
        return np.matmul(ghat, self.Jinv[elem][:, None, :, :])


def face_pattern(mesh):
    """BSR pattern: diagonal plus face neighbours, columns sorted."""
    ptr, idx = mesh.adjacency()
    ne = mesh.n_elem
    rows = np.concatenate([np.arange(ne), np.repeat(np.arange(ne), np.diff(ptr))])
    cols = np.concatenate([np.arange(ne), idx.astype(np.int64)])
    return _pattern_from_pairs(ne, rows, cols)


def _pattern_from_pairs(ne, rows, cols):
    key = np.unique(rows.astype(np.int64) * ne + cols.astype(np.int64))
    r, c = key // ne, key % ne
    row_ptr = np.zeros(ne + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), c.astype(np.int32)


def _block_positions(row_ptr, col_idx, rows, cols):
    """Index into the BSR block list of blocks (rows[i], cols[i]); all must exist."""
    ne = len(row_ptr) - 1
    key = np.repeat(np.arange(ne, dtype=np.int64), np.diff(row_ptr)) * ne + col_idx
    q = rows.astype(np.int64) * ne + cols.astype(np.int64)
    pos = np.searchsorted(key, q)
    assert np.all(key[pos] == q), "block not in pattern"
    return pos


class BSR:
    """Host block-sparse matrix: square blocks of size nb, row-major blocks."""

    def __init__(self, row_ptr, col_idx, vals):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.vals = np.ascontiguousarray(vals, dtype=np.float64)
        self.nb = self.vals.shape[1]

    @property
    def n_brow(self):
        return len(self.row_ptr) - 1

    @property
    def nnzb(self):
        return len(self.col_idx)

    @property
    def n(self):
        return self.n_brow * self.nb

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.bsr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n)).tocsr()


# ----------------------------------------------------------------------------
# SIPG
# ----------------------------------------------------------------------------

def assemble_sipg(mesh, p, penalty=10.0, chunk=200_000, log=None):
    """SIPG stiffness for -Laplace(u) = f, homogeneous Dirichlet on the boundary.
    log: optional callable given a progress message per chunk of faces."""
    dim = mesh.dim
    basis = SimplexBasis(dim, p)
    nb = basis.nb
    geo = _Geo(mesh)
    row_ptr, col_idx = face_pattern(mesh)
    vals = np.zeros((len(col_idx), nb, nb))
    ne = mesh.n_elem
    dpos = _block_positions(row_ptr, col_idx, np.arange(ne), np.arange(ne))

    # volume term: int_K grad(phi_i) . grad(phi_j)
    rule = gauss_triangle if dim == 2 else gauss_tet
    xq, wq = rule(max(p, 1))
    gh = basis.grad(xq)  # (q, nb, d)
    S = np.einsum("q,qia,qjb->abij", wq, gh, gh)
    Mt = np.einsum("eac,ebc->eab", geo.Jinv, geo.Jinv)  # J^-1 J^-T
    d2 = dim * dim
    vals[dpos] += np.abs(geo.detJ)[:, None, None] * (Mt.reshape(-1, d2) @ S.reshape(d2, -1)).reshape(-1, nb, nb)

    sig0 = penalty * p * p
    nqf = p + 1
    F = mesh.int_faces
    for s in range(0, len(F), chunk):
        if log:
            log(f"SIPG interior faces {s}/{len(F)}")
        f = F[s:s + chunk]
        ep, fp, em, fm = f[:, 0], f[:, 1], f[:, 2], f[:, 3]
        fv, n, meas = _face_geometry(mesh, ep, fp)
        x, w = _face_points(fv, dim, nqf)
        hF = np.minimum(geo.vol[ep], geo.vol[em]) / meas
        sig = sig0 / hF
        vP = basis.eval(geo.to_ref(ep, x))
        vM = basis.eval(geo.to_ref(em, x))
        dnP = np.einsum("fqid,fd->fqi", geo.phys_grad(ep, basis.grad(geo.to_ref(ep, x))), n)
        dnM = np.einsum("fqid,fd->fqi", geo.phys_grad(em, basis.grad(geo.to_ref(em, x))), n)
        vals_f = {}
        sides = {"P": (vP, dnP, 1.0), "M": (vM, dnM, -1.0)}
        for sname, (vs, dns, cs) in sides.items():        # test side (rows)
            for tname, (vt, dnt, ct) in sides.items():    # trial side (cols)
                blk = (-0.5 * cs * _wgram(w, vs, dnt)
                       - 0.5 * ct * _wgram(w, dns, vt)
                       + cs * ct * sig[:, None, None] * _wgram(w, vs, vt))
                vals_f[sname + tname] = blk
        vals[_block_positions(row_ptr, col_idx, ep, em)] = vals_f["PM"]
        vals[_block_positions(row_ptr, col_idx, em, ep)] = vals_f["MP"]
        for lf in range(dim + 1):
            m = fp == lf
            vals[dpos[ep[m]]] += vals_f["PP"][m]
            m = fm == lf
            vals[dpos[em[m]]] += vals_f["MM"][m]

    B = mesh.bnd_faces
    eb, fb = B[:, 0], B[:, 1]
    fv, n, meas = _face_geometry(mesh, eb, fb)
    x, w = _face_points(fv, dim, nqf)
    sig = sig0 / (geo.vol[eb] / meas)
    v = basis.eval(geo.to_ref(eb, x))
    dn = np.einsum("fqid,fd->fqi", geo.phys_grad(eb, basis.grad(geo.to_ref(eb, x))), n)
    blk = -_wgram(w, v, dn) - _wgram(w, dn, v) + sig[:, None, None] * _wgram(w, v, v)
    for lf in range(dim + 1):
        m = fb == lf
        vals[dpos[eb[m]]] += blk[m]
    return BSR(row_ptr, col_idx, vals)


# ----------------------------------------------------------------------------
# LDG (switch along beta, penalty on boundary faces only) + upwind convection
# ----------------------------------------------------------------------------

def assemble_ldg_upwind(mesh, p, beta, eps, penalty=10.0):
    """LDG diffusion (scaled by eps) plus upwind convection for
    -eps Laplace(u) + beta . grad(u) = f, homogeneous Dirichlet data.

    Lifted gradient q(u) on K:  (q, tau)_K = (grad u, tau)_K + sum_F <u_hat - u_K, tau.n_K>_F,
    with u_hat taken from the face's 'switch' element (the one whose outward
    normal has beta.n >= 0, i.e. the upwind side) on interior faces and u_hat = 0
    on the boundary.  The diffusion form is sum_K (q(u), q(v))_K plus a penalty
    on boundary faces: the LDG primal form with q_hat taken from the opposite side.
    """
    import scipy.sparse as sp
    dim = mesh.dim
    basis = SimplexBasis(dim, p)
    nb = basis.nb
    geo = _Geo(mesh)
    ne = mesh.n_elem
    n = ne * nb
    beta = np.asarray(beta, dtype=np.float64)

    rule = gauss_triangle if dim == 2 else gauss_tet
    xq, wq = rule(p + 1)
    phi = basis.eval(xq)              # (q, nb)
    gh = basis.grad(xq)               # (q, nb, d)
    absdet = np.abs(geo.detJ)
    # element-local gradient operator in the orthonormal basis: coefficient of
    # component a of q on K: G_a = (1/|detJ|) * int_K dphi_j/dx_a phi_i
    gphys = np.einsum("eba,qib->eqia", geo.Jinv, gh)            # (ne, q, nb, d)
    Gloc = np.einsum("q,qi,eqja->eaij", wq, phi, gphys)         # int_ref -> times |detJ| / |detJ|
    # q_a = M^-1 (...) ; M = |detJ| I, integrals carry |detJ| -> cancels for volume part
    rows, cols, data = [], [], []
    elem_dofs = np.arange(n).reshape(ne, nb)
    # volume part of the lifted gradient, for each component a
    Gblocks = [[] for _ in range(dim)]  # list of (row elem, col elem, block (ne, nb, nb))
    for a in range(dim):
        Gblocks[a].append((np.arange(ne), np.arange(ne), Gloc[:, a]))

    nqf = p + 1
    F = mesh.int_faces
    ep, fp, em, fm = F[:, 0], F[:, 1], F[:, 2], F[:, 3]
    fv, nrm, meas = _face_geometry(mesh, ep, fp)
    x, w = _face_points(fv, dim, nqf)
    vP = basis.eval(geo.to_ref(ep, x))
    vM = basis.eval(geo.to_ref(em, x))
    bn = nrm @ beta
    plus_up = bn >= 0.0  # switch side = upwind element (beta leaves through its face)
    # for the non-switch element K' with outward normal n', contribution
    # (1/|detJ_K'|) <u_s - u_K', tau . n'>  for tau = phi_i e_a
    for which in (0, 1):
        if which == 0:   # switch = plus side, K' = minus side, n' = -n
            m = plus_up
            es, vs_, ek, vk_, nk = ep[m], vP[m], em[m], vM[m], -nrm[m]
        else:            # switch = minus side, K' = plus side, n' = n
            m = ~plus_up
            es, vs_, ek, vk_, nk = em[m], vM[m], ep[m], vP[m], nrm[m]
        wk = w[m] / absdet[ek][:, None]
        for a in range(dim):
            # tau_i = phi_i^{K'} e_a ; test row on K', trial on switch element / K'
            b_s = _wgram(wk * nk[:, a][:, None], vk_, vs_)
            b_k = -_wgram(wk * nk[:, a][:, None], vk_, vk_)
            Gblocks[a].append((ek, es, b_s))
            Gblocks[a].append((ek, ek, b_k))
    B = mesh.bnd_faces
    eb, fb = B[:, 0], B[:, 1]
    fvb, nb_, measb = _face_geometry(mesh, eb, fb)
    xb, wb = _face_points(fvb, dim, nqf)
    vb = basis.eval(geo.to_ref(eb, xb))
    wkb = wb / absdet[eb][:, None]
    for a in range(dim):
        b_k = -_wgram(wkb * nb_[:, a][:, None], vb, vb)
        Gblocks[a].append((eb, eb, b_k))

    def blocks_to_sparse(blist):
        R, C, D = [], [], []
        for (re, ce, blk) in blist:
            ii = elem_dofs[re][:, :, None].repeat(nb, 2)
            jj = elem_dofs[ce][:, None, :].repeat(nb, 1)
            R.append(ii.ravel()); C.append(jj.ravel()); D.append(blk.ravel())
        return sp.csr_matrix((np.concatenate(D), (np.concatenate(R), np.concatenate(C))), shape=(n, n))

    Mdiag = sp.diags(np.repeat(absdet, nb))
    Adiff = sp.csr_matrix((n, n))
    for a in range(dim):
        Ga = blocks_to_sparse(Gblocks[a])
        Adiff = Adiff + (Ga.T @ Mdiag @ Ga)
    # boundary penalty (minimal dissipation: boundary faces only)
    sigb = penalty * p * p / (geo.vol[eb] / measb)
    pen = sigb[:, None, None] * _wgram(wb, vb, vb)
    Apen = blocks_to_sparse([(eb, eb, pen)])

    # upwind convection: -(u, beta.grad v)_K + <beta.n u_up, [v]>
    conv_vol = -np.einsum("q,eqja,a,qi->eij", wq, gphys, beta, phi) * absdet[:, None, None]
    conv_vol = np.transpose(conv_vol, (0, 2, 1))  # row = test (uses grad of test)
    cblocks = [(np.arange(ne), np.arange(ne), conv_vol)]
    # interior faces: flux beta.n u_up with n = n_plus; test v+ gets +, v- gets -
    up_is_plus = bn >= 0
    for up in (True, False):
        m = up_is_plus == up
        eu = ep[m] if up else em[m]
        vu = vP[m] if up else vM[m]
        fl = w[m] * bn[m][:, None]
        cblocks.append((ep[m], eu, _wgram(fl, vP[m], vu)))
        cblocks.append((em[m], eu, -_wgram(fl, vM[m], vu)))
    # boundary: outflow carries u, inflow carries 0
    bnb = nb_ @ beta
    out = bnb > 0
    cblocks.append((eb[out], eb[out], _wgram(wb[out] * bnb[out][:, None], vb[out], vb[out])))
    Aconv = blocks_to_sparse(cblocks)

    A = (eps * Adiff + eps * Apen + Aconv).tocsr()
    return csr_to_bsr(A, nb, ne)


def csr_to_bsr(A, nb, ne):
    """Dof-level CSR -> BSR with the block pattern of all structurally coupled element pairs."""
    A = A.tocoo()
    br, bc = A.row // nb, A.col // nb
    row_ptr, col_idx = _pattern_from_pairs(ne, np.concatenate([br, np.arange(ne)]),
                                           np.concatenate([bc, np.arange(ne)]))
    pos = _block_positions(row_ptr, col_idx, br, bc)
    vals = np.zeros((len(col_idx), nb, nb))
    np.add.at(vals, (pos, A.row % nb, A.col % nb), A.data)
    return BSR(row_ptr, col_idx, vals)


# ----------------------------------------------------------------------------
# right-hand sides and errors (manufactured solutions)
# ----------------------------------------------------------------------------

def load_vector(mesh, p, f, nq=None):
    """b_i = int f phi_i, for f a callable on (N, d) physical points."""
    basis = SimplexBasis(mesh.dim, p)
    geo = _Geo(mesh)
    rule = gauss_triangle if mesh.dim == 2 else gauss_tet
    xq, wq = rule(nq or p + 4)
    phi = basis.eval(xq)
    x = geo.v0[:, None, :] + np.einsum("eab,qb->eqa", geo.J, xq)
    fx = f(x.reshape(-1, mesh.dim)).reshape(x.shape[:2])
    return (np.abs(geo.detJ)[:, None] * np.einsum("q,eq,qi->ei", wq, fx, phi)).ravel()


def l2_error(mesh, p, coef, u, nq=None):
    basis = SimplexBasis(mesh.dim, p)
    geo = _Geo(mesh)
    rule = gauss_triangle if mesh.dim == 2 else gauss_tet
    xq, wq = rule(nq or p + 4)
    phi = basis.eval(xq)
    x = geo.v0[:, None, :] + np.einsum("eab,qb->eqa", geo.J, xq)
    ux = u(x.reshape(-1, mesh.dim)).reshape(x.shape[:2])
    uh = np.einsum("qi,ei->eq", phi, coef.reshape(mesh.n_elem, -1))
    return np.sqrt(np.sum(np.abs(geo.detJ)[:, None] * wq[None, :] * (uh - ux) ** 2))
