"""Pins for the oracle's Galerkin P0 single layer entries.

* coincident pairs: the angular reduction against an independent brute force (outer
  collapsed rule, inner Duffy split at the outer point, both at high order, written here
  in numpy) and its convergence in the number of angular points;
* unit-sphere row sums sum_j V_ij(s) vs A_i (1 - e^{-2s}) / (2s), error ~h^2;
* symmetry V_ij = V_ji up to the quadrature error, shrinking as n_G grows;
* tier selection (coincident / common edge / common vertex / distance) recomputed.
"""
import numpy as np
import pytest

from inputs import cube_mesh, icosphere_mesh, lshape_mesh
from oracle.entries import Geometry
from oracle.galerkin import galerkin_entries


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1), 0.5 * w


def _collapsed(a, b, c, n):
    x, w = _gl01(n)
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    U, V, W = U.ravel(), V.ravel(), (WU * WV).ravel()
    two_area = np.linalg.norm(np.cross(b - a, c - b))
    pts = a[None] + U[:, None] * (b - a)[None] + (U * V)[:, None] * (c - b)[None]
    return pts, W * U * two_area


def _clip_area(P, Q):
    """Area of the intersection of two convex counter-clockwise polygons (Sutherland-
    Hodgman clipping + shoelace)."""
    out = [tuple(p) for p in P]
    for k in range(len(Q)):
        a, b = np.array(Q[k]), np.array(Q[(k + 1) % len(Q)])
        inp, out = out, []
        if not inp:
            break
        side = lambda p: (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
        for i in range(len(inp)):
            cur, prv = np.array(inp[i]), np.array(inp[i - 1])
            sc, sp = side(cur), side(prv)
            if sc >= 0:
                if sp < 0:
                    t = sp / (sp - sc)
                    out.append(tuple(prv + t * (cur - prv)))
                out.append(tuple(cur))
            elif sp >= 0:
                t = sp / (sp - sc)
                out.append(tuple(prv + t * (cur - prv)))
    if len(out) < 3:
        return 0.0
    xs = np.array([p[0] for p in out])
    ys = np.array([p[1] for p in out])
    return 0.5 * abs(np.dot(xs, np.roll(ys, -1)) - np.dot(ys, np.roll(xs, -1)))


def _overlap_integral(a, b, c, s):
    """V = int k(z) area(T cap (T + z)) dz in polar coordinates, the overlap area from
    polygon clipping, both integrals adaptive (independent of the barycentric form)."""
    from scipy import integrate
    f1 = (b - a) / np.linalg.norm(b - a)
    nrm = np.cross(b - a, c - a)
    f2 = np.cross(nrm / np.linalg.norm(nrm), f1)
    T = [np.array([np.dot(p - a, f1), np.dot(p - a, f2)]) for p in (a, b, c)]
    diam = max(np.linalg.norm(T[i] - T[j]) for i in range(3) for j in range(3))
    breaks = []
    for i in range(3):
        e = T[(i + 1) % 3] - T[i]
        th = np.arctan2(e[1], e[0]) % (2 * np.pi)
        breaks += [th, (th + np.pi) % (2 * np.pi)]

    def inner(theta, part):
        d = np.array([np.cos(theta), np.sin(theta)])

        def f(rho):
            area = _clip_area(T, [p + rho * d for p in T])
            v = np.exp(-s * rho) / (4 * np.pi) * area
            return v.real if part == 0 else v.imag
        return integrate.quad(f, 0.0, diam, epsabs=1e-14, epsrel=1e-11, limit=200)[0]

    vals = []
    for part in (0, 1):
        vals.append(integrate.quad(lambda th: inner(th, part), 0.0, 2 * np.pi,
                                   points=sorted(breaks), epsabs=1e-13, epsrel=1e-10,
                                   limit=200)[0])
    return vals[0] + 1j * vals[1]


TRIS = [np.array([[0, 0, 0], [1, 0, 0], [0.3, 0.8, 0.0]]),
        np.array([[0, 0, 0], [1 / 16, 0, 0], [1 / 16, 1 / 16, 0]]),
        np.array([[0.1, 0.2, 0.3], [0.2, 0.25, 0.31], [0.12, 0.3, 0.35]])]


@pytest.mark.parametrize("tid", range(len(TRIS)))
@pytest.mark.parametrize("s", [0.0, 2.0 + 3.0j, 39.0 - 0.9j])
def test_coincident_angular_vs_brute_force(tid, s):
    v = TRIS[tid]
    g = Geometry(v, np.array([[0, 1, 2]], dtype=np.int32))
    got = galerkin_entries(g, "slp", np.array([s]), [0], [0])[0, 0]
    ref = _overlap_integral(v[0], v[1], v[2], s)
    assert abs(got - ref) <= 1e-8 * abs(ref), (got, ref)
    hi = galerkin_entries(g, "slp", np.array([s]), [0], [0], n_theta=48)[0, 0]
    assert abs(got - hi) <= 1e-12 * abs(hi)


def test_sphere_row_sums_converge():
    S = np.array([0.0, 1.0, 2.0 + 3.0j, 6.0 - 2.0j])
    with np.errstate(all="ignore"):
        ex = np.where(S == 0, 1.0, (1 - np.exp(-2 * S)) / (2 * np.where(S == 0, 1, S)))
    errs = []
    for lev in (2, 3):
        x, t = icosphere_mesh(lev)
        g = Geometry(x, t)
        M = t.shape[0]
        rows = np.arange(0, M, max(1, M // 8))
        ii = np.repeat(rows, M)
        jj = np.tile(np.arange(M), rows.shape[0])
        V = galerkin_entries(g, "slp", S, ii, jj).reshape(rows.shape[0], M, -1).sum(axis=1)
        a, b, c = x[t[:, 0]], x[t[:, 1]], x[t[:, 2]]
        A = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
        errs.append(np.abs(V / A[rows, None] - ex[None]).max(axis=0))
    errs = np.array(errs)
    assert np.all(errs[0] / errs[1] > 3.0), errs
    assert np.all(errs[1] < 3e-3), errs


def test_symmetry_improves_with_order():
    x, t = lshape_mesh(2)
    g = Geometry(x, t)
    M = t.shape[0]
    rng = np.random.default_rng(2)
    cen = (x[t[:, 0]] + x[t[:, 1]] + x[t[:, 2]]) / 3
    ii, jj = [], []
    for i in rng.choice(M, 40, replace=False):
        d = np.linalg.norm(cen - cen[i], axis=1)
        for j in np.argsort(d)[1:6]:
            ii.append(i)
            jj.append(j)
    ii, jj = np.array(ii), np.array(jj)
    s = np.array([1.0 + 2.0j, 15.0 + 10.0j])
    asym = []
    for ng in (3, 5, 9):
        a = galerkin_entries(g, "slp", s, ii, jj, n_g=ng)
        b = galerkin_entries(g, "slp", s, jj, ii, n_g=ng)
        asym.append(np.max(np.abs(a - b) / np.abs(a)))
    # measured: ~1.4e-2 (n_G = 3), ~1.5e-3 (5, the default), ~1.4e-4 (9): the outer rule
    # converges algebraically next to the shared edge / vertex
    assert asym[0] > asym[1] > asym[2], asym
    assert asym[1] < 3e-3 and asym[2] < 3e-4, asym


def test_tier_selection():
    x, t = cube_mesh(4)
    g = Geometry(x, t)
    M = t.shape[0]
    rng = np.random.default_rng(4)
    ii = rng.integers(0, M, 2000)
    jj = rng.integers(0, M, 2000)
    jj[:30] = ii[:30]
    far = (rng.random(2000) < 0.1).astype(np.int32)
    _, tier = galerkin_entries(g, "slp", np.array([1.0]), ii, jj, far, return_tier=True)
    a, b, c = x[t[:, 0]], x[t[:, 1]], x[t[:, 2]]
    cen = (a + b + c) / 3
    h = np.max(np.stack([np.linalg.norm(b - a, axis=1), np.linalg.norm(c - a, axis=1),
                         np.linalg.norm(c - b, axis=1)]), axis=0)
    shared = np.array([len(set(t[i]) & set(t[j])) for i, j in zip(ii, jj)])
    q = np.linalg.norm(cen[ii] - cen[jj], axis=1) / np.maximum(h[ii], h[jj])
    expect = np.where(q >= 4, 0, np.where(q >= 2, 1, 2))
    expect = np.where(shared == 1, 4, expect)
    expect = np.where(shared == 2, 3, expect)
    expect = np.where(far == 1, 0, expect)
    expect = np.where(ii == jj, 5, expect)
    assert np.array_equal(tier, expect)
