"""Pins for the oracle's quadrature rules: exactness on monomials (closed forms)."""
from math import factorial

import numpy as np
import pytest

from oracle import quadrature as Q


def _tri_monomial(a, b):
    # int over {x, y >= 0, x + y <= 1} of x^a y^b = a! b! / (a + b + 2)!
    return factorial(a) * factorial(b) / factorial(a + b + 2)


def test_triangle6_weights_and_points():
    p, w = Q.triangle6()
    assert p.shape == (6, 3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(p.sum(axis=1), 1.0, atol=1e-15)
    # published decimal values of the 6-point degree-4 rule (Strang-Fix / Cowper)
    assert abs(w[0] - 0.223381589678011) < 1e-14
    assert abs(w[3] - 0.109951743655322) < 1e-14
    assert abs(p[1, 0] - 0.445948490915965) < 1e-14
    assert abs(p[4, 0] - 0.091576213509771) < 1e-14


@pytest.mark.parametrize("deg", range(0, 5))
def test_triangle6_exact_to_degree_4(deg):
    p, w = Q.triangle6()
    x, y = p[:, 1], p[:, 2]   # reference triangle (0,0),(1,0),(0,1): x = l2, y = l3
    for a in range(deg + 1):
        b = deg - a
        approx = 0.5 * np.sum(w * x ** a * y ** b)
        assert abs(approx - _tri_monomial(a, b)) < 1e-15


def test_triangle6_not_exact_at_degree_6():
    p, w = Q.triangle6()
    x = p[:, 1]
    assert abs(0.5 * np.sum(w * x ** 6) - _tri_monomial(6, 0)) > 1e-6


@pytest.mark.parametrize("n", [1, 2, 4, 8, 10])
def test_gauss01_exact(n):
    x, w = Q.gauss01(n)
    for d in range(2 * n):
        assert abs(np.sum(w * x ** d) - 1.0 / (d + 1)) < 1e-14
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("n", [2, 4, 8])
def test_collapsed_rule_exact(n):
    a = np.array([0.0, 0.0, 0.0])
    b = np.array([1.0, 0.0, 0.0])
    c = np.array([0.0, 1.0, 0.0])
    pts, wts = Q.collapsed_points(a, b, c, n)
    assert abs(wts.sum() - 0.5) < 1e-15
    for deg in range(0, 2 * n - 1):
        for i in range(deg + 1):
            j = deg - i
            approx = np.sum(wts * pts[:, 0] ** i * pts[:, 1] ** j)
            assert abs(approx - _tri_monomial(i, j)) < 1e-14


def test_collapsed_rule_general_triangle_area():
    rng = np.random.default_rng(3)
    a, b, c = rng.standard_normal((3, 3))
    pts, wts = Q.collapsed_points(a, b, c, 4)
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    assert abs(wts.sum() - area) < 1e-14
    # first moments give the centroid
    cen = (wts[:, None] * pts).sum(axis=0) / wts.sum()
    assert np.allclose(cen, (a + b + c) / 3.0, atol=1e-14)
