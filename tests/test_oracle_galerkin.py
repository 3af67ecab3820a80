"""Pins for the oracle's Galerkin P0 single layer entries.

* coincident pairs: the angular reduction against an independent brute force (outer
  collapsed rule, inner Duffy split at the outer point, both at high order, written here
  in numpy) and its convergence in the number of angular points;
* unit-sphere row sums sum_j V_ij(s) vs A_i (1 - e^{-2s}) / (2s), error ~h^2;
* touching pairs (common edge, common vertex) against an independent reference written
  here: the inner integral in polar coordinates at the foot point of the outer point (radial
  integral exact, angular integral per edge by composite Gauss in the angle and in log
  arclength), the outer integral by a geometrically graded tensor Gauss rule toward the
  shared edge or vertex; coplanar, 90-degree and reentrant (270-degree) edges;
* symmetry V_ij = V_ji to 1e-8 on every touching pair of a small L-shape at the default order;
* disjoint near pairs: symmetry improving with n_G;
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


def _g01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1), 0.5 * w


def _inner_polar(X, a, b, c, s, n_phi=20, n_w=12, panels=20):
    """F(x) = int_{tau} e^{-s|x-y|} / (4 pi |x-y|) dS_y for the rows x of X.  Polar
    coordinates around the foot point p of x in the plane of tau (distance d): over the
    sub-triangle (p, v_a, v_b) the radial integral is (e^{-s d} - e^{-s R}) / (4 pi s),
    R = sqrt(rho_edge^2 + d^2); the angle is integrated per edge in arclength u from the
    foot of p on the edge line (distance h): phi = atan(u / h) for |u| <= h and log u for
    |u| > h, composite Gauss; sub-triangles on the outer side of an edge count negative."""
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm)
    d = (X - a) @ nrm
    P = X - d[:, None] * nrm[None]
    d = np.abs(d)
    out = np.zeros(X.shape[0], complex)
    xp, wp = _g01(n_phi)
    xw, ww = _g01(n_w)
    e_sd = np.exp(-s * d)

    def G(u, h):
        R = np.sqrt(u * u + h * h + d[:, None] ** 2)
        return (e_sd[:, None] - np.exp(-s * R)) / (4 * np.pi * s)

    for va, vb in ((a, b), (b, c), (c, a)):
        ev = vb - va
        ell = np.linalg.norm(ev)
        e = ev / ell
        t = (P - va) @ e
        h = np.linalg.norm(va[None] + t[:, None] * e[None] - P, axis=1)
        side = np.sign(np.cross(ev, P - va) @ nrm)
        ua, ub = -t, ell - t
        ok = h > 0
        hh = np.where(ok, h, 1.0)
        tot = np.zeros(X.shape[0], complex)
        for sgn in (-1.0, 1.0):
            lo = np.clip(np.where(sgn > 0, ua, -ub), 0, None)
            hi = np.clip(np.where(sgn > 0, ub, -ua), 0, None)
            p0 = np.arctan(np.minimum(lo, hh) / hh)
            p1 = np.arctan(np.minimum(hi, hh) / hh)
            ph = p0[:, None] + (p1 - p0)[:, None] * xp[None]
            tot += np.sum(G(sgn * hh[:, None] * np.tan(ph), hh[:, None]) * wp[None]
                          * (p1 - p0)[:, None], axis=1)
            l0 = np.log(np.maximum(lo, hh))
            l1 = np.maximum(np.log(np.maximum(hi, hh)), l0)
            for k in range(panels):
                q0 = l0 + (l1 - l0) * k / panels
                q1 = l0 + (l1 - l0) * (k + 1) / panels
                u = np.exp(q0[:, None] + (q1 - q0)[:, None] * xw[None])
                tot += np.sum(G(sgn * u, hh[:, None]) * hh[:, None] * u / (hh[:, None] ** 2 + u * u)
                              * ww[None] * (q1 - q0)[:, None], axis=1)
        out += np.where(ok, side * tot, 0.0)
    return out


def _graded(n, K, sigma, at0, at1):
    brk = [0.0, 1.0]
    if at0:
        brk += [sigma ** k * (0.5 if at1 else 1.0) for k in range(1, K + 1)]
    if at1:
        brk += [1 - sigma ** k * 0.5 for k in range(1, K + 1)] + [0.5]
    brk = np.unique(brk)
    x, w = _g01(n)
    return (np.concatenate([lo + (hi - lo) * x for lo, hi in zip(brk[:-1], brk[1:])]),
            np.concatenate([(hi - lo) * w for lo, hi in zip(brk[:-1], brk[1:])]))


def _touching_reference(P0, P1, P2, tau_j, s, edge, n=10, K=12, sigma=0.15):
    """int_{tau_i} F dS_x with tau_i = (P0, P1, P2) in collapsed coordinates at P0
    (x = P0 + u (P1 - P0) + u v (P2 - P1)); the shared vertex is P0, the shared edge P0 P1
    (v = 0); the rule is graded toward u = 0 (and u = 1, v = 0 for an edge)."""
    u, wu = _graded(n, K, sigma, True, edge)
    v, wv = _graded(n, K if edge else 0, sigma, edge, False)
    U, V = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    U, V, W = U.ravel(), V.ravel(), (WU * WV).ravel()
    two = np.linalg.norm(np.cross(P1 - P0, P2 - P1))
    X = P0[None] + U[:, None] * (P1 - P0)[None] + (U * V)[:, None] * (P2 - P1)[None]
    tot = 0.0
    for k0 in range(0, X.shape[0], 4000):
        sl = slice(k0, k0 + 4000)
        tot += np.sum(_inner_polar(X[sl], *tau_j, s) * W[sl] * U[sl] * two)
    return tot


_H = 1.0 / 16
_TV = np.array([[0, 0, 0], [_H, 0, 0], [_H, _H, 0], [0, _H, 0], [0, 0, _H], [_H, 0, _H],
                [2 * _H, _H, 0], [_H, 0, -_H], [0.5 * _H, 0.3 * _H, 0.8 * _H], [-_H, 0, 0]], float)
_TT = np.array([[0, 1, 2], [0, 2, 3], [1, 0, 4], [2, 6, 1], [0, 1, 7], [1, 0, 8],
                [3, 9, 0]], dtype=np.int32)
# (i, j, what, s): right-isosceles grid triangles as in the cube and L-shape meshes
_TOUCH = [(0, 1, "edge coplanar", 2.0 + 3.0j), (0, 2, "edge 90 degrees", 38.0 - 12.0j),
          (2, 4, "edge 270 degrees (reentrant)", 20.0 + 19.0j),
          (0, 5, "edge, tilted third vertex", 1.0 + 0.5j),
          (0, 6, "vertex coplanar", 38.0 - 12.0j), (2, 6, "vertex 90 degrees", 2.0 + 3.0j),
          (4, 3, "vertex opposite faces", 20.0 - 19.0j)]


@pytest.mark.parametrize("case", range(len(_TOUCH)))
def test_touching_pairs_vs_adaptive_reference(case):
    i, j, what, s = _TOUCH[case]
    g = Geometry(_TV, _TT)
    got, tier = galerkin_entries(g, "slp", np.array([s]), [i], [j], return_tier=True)
    shared = [a for a in range(3) if _TT[i][a] in _TT[j]]
    vi = _TV[_TT[i]]
    if len(shared) == 2:
        assert tier[0] == 3, what
        P0, P1, P2 = vi[shared[0]], vi[shared[1]], vi[3 - sum(shared)]
    else:
        assert tier[0] == 4 and len(shared) == 1, what
        a = shared[0]
        P0, P1, P2 = vi[a], vi[(a + 1) % 3], vi[(a + 2) % 3]
    vj = _TV[_TT[j]]
    ref = _touching_reference(P0, P1, P2, (vj[0], vj[1], vj[2]), s, len(shared) == 2)
    assert abs(got[0, 0] - ref) <= 1e-8 * abs(ref), (what, got[0, 0], ref)


def test_touching_pairs_symmetric():
    x, t = lshape_mesh(2)
    g = Geometry(x, t)
    sets = [set(r) for r in t]
    ii, jj = [], []
    for i in range(t.shape[0]):
        for j in range(t.shape[0]):
            if i != j and sets[i] & sets[j]:
                ii.append(i)
                jj.append(j)
    s = np.array([1.0 + 2.0j, 15.0 + 10.0j, 38.0 - 12.0j])
    a, tier = galerkin_entries(g, "slp", s, ii, jj, return_tier=True)
    b = galerkin_entries(g, "slp", s, jj, ii)
    assert set(np.unique(tier)) == {3, 4}
    assert np.max(np.abs(a - b) / np.abs(a)) <= 1e-8


def test_symmetry_improves_with_order():
    x, t = lshape_mesh(2)
    g = Geometry(x, t)
    M = t.shape[0]
    rng = np.random.default_rng(2)
    cen = (x[t[:, 0]] + x[t[:, 1]] + x[t[:, 2]]) / 3
    sets = [set(r) for r in t]
    ii, jj = [], []
    for i in rng.choice(M, 60, replace=False):
        d = np.linalg.norm(cen - cen[i], axis=1)
        for j in np.argsort(d)[1:16]:
            if not sets[i] & sets[j]:
                ii.append(i)
                jj.append(j)
    ii, jj = np.array(ii), np.array(jj)
    s = np.array([1.0 + 2.0j, 15.0 + 10.0j])
    asym = []
    for ng in (3, 5, 9):
        a = galerkin_entries(g, "slp", s, ii, jj, n_g=ng)
        b = galerkin_entries(g, "slp", s, jj, ii, n_g=ng)
        asym.append(np.max(np.abs(a - b) / np.abs(a)))
    _, tier = galerkin_entries(g, "slp", s[:1], ii, jj, return_tier=True)
    assert set(np.unique(tier)) <= {0, 1, 2} and 2 in tier
    assert asym[0] > asym[1] > asym[2], asym


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
