"""Quadrature rules used by the oracle (test infrastructure only).

The paper integrates the load vector and the error norms with an unspecified
"high-order numerical integration" (Sec. 4).  The oracle reads this as tensor
Gauss-Legendre in time and a collapsed (Duffy) Gauss rule on each triangle.
The Gauss-Legendre nodes come from numpy's library routine.
"""
import numpy as np


def gauss_legendre(m):
    """m-point Gauss-Legendre rule on [0, 1]: (points, weights).

    Exact for polynomials of degree <= 2m-1."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(m):
    """Collapsed Gauss rule on the reference triangle {x, y >= 0, x + y <= 1}.

    The square (u, v) in [0,1]^2 is mapped by x = u, y = v (1 - u), whose
    Jacobian is (1 - u).  With m Gauss-Legendre points per direction the
    rule integrates every polynomial of total degree <= 2m - 2 exactly.
    Returns (points (k, 2), weights (k,)) with weights summing to 1/2."""
    g, w = gauss_legendre(m)
    u, v = np.meshgrid(g, g, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    x = u.ravel()
    y = (v * (1.0 - u)).ravel()
    wt = (wu * wv * (1.0 - u)).ravel()
    return np.stack([x, y], axis=1), wt
