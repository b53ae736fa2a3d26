"""Quadrature on reference simplices (oracle; test infrastructure only).

The paper asks for quadrature that integrates every form exactly (end of
section 2.2).  Reading used here: collapsed (Stroud conical product)
Gauss-Jacobi rules; n points per collapsed direction integrate total degree
2n - 1 exactly.  Nodes and weights come from scipy.special.roots_jacobi
(Golub-Welsch), a library primitive.

Reference simplices: the unit interval [0,1], the triangle with vertices
(0,0),(1,0),(0,1), the tetrahedron with vertices 0, e1, e2, e3.
  triangle: x2 = (1+b)/2, x1 = (1+a)(1-b)/4, w = wa wb / 8,
            a ~ Gauss-Jacobi(0,0), b ~ Gauss-Jacobi(1,0)
  tet:      x3 = (1+c)/2, x2 = (1+b)(1-c)/4, x1 = (1+a)(1-b)(1-c)/8,
            w = wa wb wc / 64, c ~ Gauss-Jacobi(2,0)
"""
import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi(n, alpha, beta):
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def simplex_rule(dim, n):
    """Points [nq][dim] and weights [nq] on the reference dim-simplex
    (dim = 1, 2, 3), n points per collapsed direction."""
    if dim == 1:
        x, w = gauss_jacobi(n, 0.0, 0.0)
        return ((1.0 + x) / 2.0)[:, None], w / 2.0
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    if dim == 2:
        A, B = np.meshgrid(a, b, indexing="ij")
        WA, WB = np.meshgrid(wa, wb, indexing="ij")
        x2 = (1.0 + B) / 2.0
        x1 = (1.0 + A) * (1.0 - B) / 4.0
        pts = np.stack([x1.ravel(), x2.ravel()], -1)
        return pts, (WA * WB).ravel() / 8.0
    c, wc = gauss_jacobi(n, 2.0, 0.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    x3 = (1.0 + C) / 2.0
    x2 = (1.0 + B) * (1.0 - C) / 4.0
    x1 = (1.0 + A) * (1.0 - B) * (1.0 - C) / 8.0
    pts = np.stack([x1.ravel(), x2.ravel(), x3.ravel()], -1)
    return pts, (WA * WB * WC).ravel() / 64.0


def volume_points_per_dir(k):
    """Volume rule for the convection form: (u x u):grad v has degree 3k-1 on
    an affine simplex, so ceil(3k/2) points per direction."""
    return (3 * k + 1) // 2


def facet_points_per_dir(k):
    """Facet rule: (u.n)<u>.[[v]] has degree 3k, so ceil((3k+1)/2) points."""
    return (3 * k + 2) // 2
