"""Seeded synthetic simplex meshes (input generation only).

These stand in for the meshes of the paper's experiments (structured and
Gmsh-generated unstructured meshes of a cube, Section 5), which are not
available: split-square triangulations, jittered-grid Delaunay triangulations
of the unit square and jittered Kuhn (6-tetrahedra) subdivisions of the unit
cube.  Every mesh is returned in a canonical form:

* ``verts`` (nv, d) float64 and ``elems`` (ne, d+1) int64, every element
  positively oriented;
* elements sorted lexicographically by their (rotated) vertex lists, so the
  element order does not depend on the Delaunay library's output order.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import Delaunay


@dataclass
class Mesh:
    verts: np.ndarray
    elems: np.ndarray
    dim: int
    # filled by build_faces()
    int_faces: np.ndarray = field(default=None)   # (nf, 4): e_plus, local face, e_minus, local face
    bnd_faces: np.ndarray = field(default=None)   # (nb, 2): element, local face

    @property
    def n_elem(self):
        return len(self.elems)

    def centroids(self):
        return self.verts[self.elems].mean(axis=1)

    def volumes(self):
        J = self.jacobians()
        fact = 2.0 if self.dim == 2 else 6.0
        return np.abs(np.linalg.det(J)) / fact

    def jacobians(self):
        v = self.verts[self.elems]
        return np.stack([v[:, k + 1] - v[:, 0] for k in range(self.dim)], axis=2)  # (ne, d, d) columns

    def adjacency(self):
        """Face-neighbour graph of the elements as CSR (int32 ptr, int32 idx), sorted."""
        ne = self.n_elem
        a = np.concatenate([self.int_faces[:, 0], self.int_faces[:, 2]])
        b = np.concatenate([self.int_faces[:, 2], self.int_faces[:, 0]])
        order = np.lexsort((b, a))
        a, b = a[order], b[order]
        ptr = np.zeros(ne + 1, dtype=np.int64)
        np.add.at(ptr, a + 1, 1)
        return np.cumsum(ptr).astype(np.int32), b.astype(np.int32)


def _canonicalise(verts, elems, dim):
    elems = np.asarray(elems, dtype=np.int64).copy()
    v = verts[elems]
    J = np.stack([v[:, k + 1] - v[:, 0] for k in range(dim)], axis=2)
    neg = np.linalg.det(J) < 0
    elems[neg, 0], elems[neg, 1] = elems[neg, 1].copy(), elems[neg, 0].copy()
    if dim == 2:
        # rotate (an even permutation) so the smallest vertex id comes first
        r = np.argmin(elems, axis=1)
        idx = (r[:, None] + np.arange(3)[None, :]) % 3
        elems = np.take_along_axis(elems, idx, axis=1)
    order = np.lexsort(elems.T[::-1])
    return elems[order]


def build_faces(mesh):
    """Match the faces (face f of an element is opposite its local vertex f)."""
    d = mesh.dim
    ne = mesh.n_elem
    nf_loc = d + 1
    loc = [[v for v in range(nf_loc) if v != f] for f in range(nf_loc)]
    keys = np.concatenate([np.sort(mesh.elems[:, loc[f]], axis=1) for f in range(nf_loc)], axis=0)
    owner = np.tile(np.arange(ne), nf_loc)
    lface = np.repeat(np.arange(nf_loc), ne)
    order = np.lexsort(keys.T[::-1])
    ks = keys[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    first = np.nonzero(same)[0]
    paired = np.zeros(len(ks), dtype=bool)
    paired[first] = True
    paired[first + 1] = True
    i1, i2 = order[first], order[first + 1]
    e1, e2 = owner[i1], owner[i2]
    swap = e1 > e2
    ep = np.where(swap, e2, e1)
    em = np.where(swap, e1, e2)
    fp = np.where(swap, lface[i2], lface[i1])
    fm = np.where(swap, lface[i1], lface[i2])
    intf = np.stack([ep, fp, em, fm], axis=1)
    intf = intf[np.lexsort((intf[:, 2], intf[:, 0]))]
    bi = order[~paired]
    bnd = np.stack([owner[bi], lface[bi]], axis=1)
    bnd = bnd[np.lexsort((bnd[:, 1], bnd[:, 0]))]
    mesh.int_faces, mesh.bnd_faces = intf.astype(np.int64), bnd.astype(np.int64)
    return mesh


def split_square(nx):
    """nx*nx cells of the unit square, each split along its (i,j)->(i+1,j+1) diagonal."""
    s = np.linspace(0.0, 1.0, nx + 1)
    X, Y = np.meshgrid(s, s, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    j, i = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    v00 = (j * (nx + 1) + i).ravel()
    v10, v01 = v00 + 1, v00 + nx + 1
    v11 = v01 + 1
    tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    return build_faces(Mesh(verts, _canonicalise(verts, tris, 2), 2))


def jittered_delaunay(side, jitter=0.25, seed=0):
    """Delaunay triangulation of a side*side grid of the unit square whose interior
    points are moved by U(-jitter*h, jitter*h) per coordinate (boundary fixed)."""
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, 1.0, side)
    h = 1.0 / (side - 1)
    X, Y = np.meshgrid(s, s, indexing="xy")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    interior = (pts[:, 0] > 0) & (pts[:, 0] < 1) & (pts[:, 1] > 0) & (pts[:, 1] < 1)
    pts = pts + rng.uniform(-jitter * h, jitter * h, size=pts.shape) * interior[:, None]
    tri = Delaunay(pts, qhull_options="Qbb Qc Qz Q12")
    return build_faces(Mesh(pts, _canonicalise(pts, tri.simplices, 2), 2))


def kuhn_cube(n, jitter=0.2, seed=0):
    """n^3 cells of the unit cube, each split into 6 Kuhn tetrahedra around its main
    diagonal; interior vertices moved by U(-jitter*h, jitter*h) per coordinate."""
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, 1.0, n + 1)
    Z, Y, X = np.meshgrid(s, s, s, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    interior = np.all((verts > 0) & (verts < 1), axis=1)
    h = 1.0 / n
    verts = verts + rng.uniform(-jitter * h, jitter * h, size=verts.shape) * interior[:, None]
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = (k * (n + 1) ** 2 + j * (n + 1) + i).ravel()
    step = np.array([1, n + 1, (n + 1) ** 2])
    tets = []
    for perm in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
        v0 = base
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v2 + step[perm[2]]
        tets.append(np.stack([v0, v1, v2, v3], 1))
    return build_faces(Mesh(verts, _canonicalise(verts, np.concatenate(tets), 3), 3))
