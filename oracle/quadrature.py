"""Oracle: quadrature rules (test infrastructure only).

The paper treats regular integrals with Gauss rules chosen by a distance heuristic and
the collocation singularity with a Duffy transformation (Sec. 3, spatial
discretisation), without giving orders.  The orders used here are a reading of that
passage:

* 6-point symmetric triangle rule of degree 4 (Strang-Fix / Cowper), from its closed
  form in radicals;
* Gauss-Legendre rules on [0, 1] (numpy's ``leggauss`` as the library primitive);
* the collapsed ("Duffy square") rule on a triangle: y(u, v) = a + u (b - a) + u v (c - b)
  with Jacobian 2 A u, Gauss-Legendre in u and v.

Pins: exactness on monomials (tests/test_oracle_quadrature.py).
"""
from __future__ import annotations

import numpy as np


def triangle6():
    """Barycentric points (l1, l2, l3) and weights (summing to 1) of the 6-point rule."""
    r10 = np.sqrt(10.0)
    root = np.sqrt(38.0 - 44.0 * np.sqrt(2.0 / 5.0))
    a1 = (8.0 - r10 + root) / 18.0
    a2 = (8.0 - r10 - root) / 18.0
    wr = np.sqrt(213125.0 - 53320.0 * r10)
    w1 = (620.0 + wr) / 3720.0
    w2 = (620.0 - wr) / 3720.0
    pts, wts = [], []
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        for p in ((b, a, a), (a, b, a), (a, a, b)):
            pts.append(p)
            wts.append(w)
    return np.array(pts), np.array(wts)


def gauss01(n):
    """n-point Gauss-Legendre on [0, 1]: (nodes, weights)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def collapsed_points(a, b, c, n):
    """Physical points and weights of the n x n collapsed rule on triangle (a, b, c)
    with the collapsed edge at vertex a."""
    x, w = gauss01(n)
    e1 = b - a
    e2 = c - b
    two_area = np.linalg.norm(np.cross(e1, e2))
    pts, wts = [], []
    for iu in range(n):
        for iv in range(n):
            u, v = x[iu], x[iv]
            pts.append(a + u * e1 + u * v * e2)
            wts.append(w[iu] * w[iv] * u * two_area)
    return np.array(pts), np.array(wts)
