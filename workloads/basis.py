"""Orthonormal polynomial bases of total degree <= p on the reference simplex.

The basis is the monomial basis orthonormalised in the L2 inner product of
the reference element (Cholesky of the monomial Gram matrix, computed with an
exact quadrature rule).  On an affine element K the element mass matrix is then
``|det J_K| * I``, so the mass matrix is trivially absorbed into the right-hand
side as the DG formulation in the paper does (Section 2, eq:Auf).
"""
import itertools

import numpy as np

from .quadrature import gauss_tet, gauss_triangle


class SimplexBasis:
    def __init__(self, dim, p):
        self.dim, self.p = dim, p
        self.exps = np.array(
            [e for tot in range(p + 1) for e in itertools.product(range(tot + 1), repeat=dim) if sum(e) == tot],
            dtype=np.int64,
        )
        self.nb = len(self.exps)
        rule = gauss_triangle if dim == 2 else gauss_tet
        xq, wq = rule(p + 2)
        M = self._monomials(xq)  # (q, nb)
        G = (M * wq[:, None]).T @ M
        L = np.linalg.cholesky(G)
        self.C = np.linalg.inv(L)  # phi = C @ monomials

    def _monomials(self, xi):
        out = np.ones(xi.shape[:-1] + (len(self.exps),))
        for k, e in enumerate(self.exps):
            for d in range(self.dim):
                if e[d]:
                    out[..., k] *= xi[..., d] ** e[d]
        return out

    def _monomial_grads(self, xi):
        out = np.zeros(xi.shape[:-1] + (len(self.exps), self.dim))
        for k, e in enumerate(self.exps):
            for d in range(self.dim):
                if e[d] == 0:
                    continue
                term = np.full(xi.shape[:-1], float(e[d]))
                for dd in range(self.dim):
                    pw = e[dd] - (1 if dd == d else 0)
                    if pw:
                        term = term * xi[..., dd] ** pw
                out[..., k, d] = term
        return out

    def eval(self, xi):
        """Basis values at reference points xi (..., dim) -> (..., nb)."""
        return self._monomials(xi) @ self.C.T

    def grad(self, xi):
        """Reference gradients at xi (..., dim) -> (..., nb, dim)."""
        g = self._monomial_grads(xi)
        return np.matmul(self.C, g)
