"""Quadrature rules on the reference simplices (input generation only).

Collapsed-coordinate (Duffy) tensor rules built from Gauss-Legendre and
Gauss-Jacobi nodes.  A rule with ``n`` points per direction integrates
polynomials of total degree ``2n - 1`` exactly.

Reference triangle: vertices (0,0), (1,0), (0,1); area 1/2.
Reference tetrahedron: vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1); volume 1/6.
"""
import numpy as np
from scipy.special import roots_jacobi, roots_legendre


def gauss_line(n):
    """Gauss-Legendre rule on [0, 1]: returns (t, w), sum(w) = 1."""
    x, w = roots_legendre(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_triangle(n):
    """Collapsed rule on the reference triangle: returns (xi (q,2), w (q,))."""
    a, wa = roots_legendre(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)  # weight (1-b) absorbs the Duffy Jacobian
    A, B = np.meshgrid(a, b, indexing="ij")
    WA, WB = np.meshgrid(wa, wb, indexing="ij")
    xi = 0.25 * (1.0 + A) * (1.0 - B)
    eta = 0.5 * (1.0 + B)
    w = WA * WB / 8.0
    return np.stack([xi.ravel(), eta.ravel()], axis=1), w.ravel()


def gauss_tet(n):
    """Collapsed rule on the reference tetrahedron: returns (xi (q,3), w (q,))."""
    a, wa = roots_legendre(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    c, wc = roots_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    x = 0.125 * (1.0 + A) * (1.0 - B) * (1.0 - C)
    y = 0.25 * (1.0 + B) * (1.0 - C)
    z = 0.5 * (1.0 + C)
    w = WA * WB * WC / 64.0
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), w.ravel()
