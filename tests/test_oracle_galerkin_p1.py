"""Pins of the oracle's Galerkin P1 operators of the Neumann problem (eq. bie_semi_neum):
the hypersingular operator D after integration by parts and the adjoint double layer K'.

* regularising maps: every map family (identical triangles, shared edge, shared vertex)
  integrates monomials of the reference coordinates exactly (it covers the pair of reference
  triangles once);
* touching pairs: summed over the weights (sum_ab lambda_a lambda_b = 1) the local matrices
  of G_s equal the P0 Galerkin single layer of the same pair, which the other oracle
  computes with closed-form radial integrals (pinned there to 1e-10);
* disjoint pairs take the same rules as that oracle: the sums agree to rounding;
* the dG/dn_x local matrices of separated pairs against a brute-force midpoint rule;
* D annihilates constants at s = 0 (the curls of the hat functions sum to zero);
* unit sphere: sum_ij D_ij -> 4 pi D1(s) and sum_ij K'_ij -> 4 pi K'1(s), the closed forms of
  the operators applied to a constant density (modified spherical Bessel functions), at
  second order in h."""
import numpy as np
import pytest

from inputs import icosphere_mesh, lshape_mesh
from oracle.entries import Geometry, P1Geometry
from oracle.galerkin import galerkin_entries
from oracle.galerkin_p1 import p1_galerkin_entries, pair_local, ss_monomial


@pytest.mark.parametrize("rel", [3, 2, 1])
def test_regularising_maps_integrate_monomials(rel):
    for a, b, c, d in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 2), (2, 1, 1, 3), (3, 2, 2, 1)]:
        exact = 1.0 / ((b + 1) * (a + b + 2)) / ((d + 1) * (c + d + 2))
        assert abs(ss_monomial(rel, a, b, c, d, 8) - exact) <= 1e-14, (rel, a, b, c, d)


def _touching_pairs(tri, step):
    ti, tj = [], []
    M = tri.shape[0]
    for t in range(0, M, step):
        for u in range(M):
            if len(set(tri[t]) & set(tri[u])) > 0:
                ti.append(t)
                tj.append(u)
    return np.array(ti), np.array(tj)


@pytest.mark.parametrize("mesh", ["lshape", "sphere"])
def test_touching_pairs_sum_to_p0_galerkin(mesh):
    xyz, tri = lshape_mesh(2) if mesh == "lshape" else icosphere_mesh(2)
    s = np.array([0.5, 3.0 + 2.0j, 10.0 - 5.0j])
    ti, tj = _touching_pairs(tri, max(1, tri.shape[0] // 12))
    ref = galerkin_entries(Geometry(xyz, tri), "slp", s, ti, tj, np.zeros(ti.shape[0], np.int32))
    tot = pair_local(xyz, tri, "g", s, ti, tj, n_ss=10).sum(axis=(1, 2))
    err = np.abs(tot - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert err.max() <= 1e-8, err.max()


def test_disjoint_pairs_match_p0_rules():
    xyz, tri = lshape_mesh(2)
    M = tri.shape[0]
    rng = np.random.default_rng(4)
    ti, tj = rng.integers(0, M, 600), rng.integers(0, M, 600)
    keep = np.array([len(set(tri[a]) & set(tri[b])) == 0 for a, b in zip(ti, tj)])
    ti, tj = ti[keep], tj[keep]
    far = (rng.random(ti.shape[0]) < 0.3).astype(np.int32)
    s = np.array([1.0 + 1.0j, 6.0])
    ref = galerkin_entries(Geometry(xyz, tri), "slp", s, ti, tj, far)
    tot = pair_local(xyz, tri, "g", s, ti, tj, far).sum(axis=(1, 2))
    assert np.abs(tot - ref).max() <= 1e-13 * np.abs(ref).max()


def test_dnx_local_matrices_against_brute_force():
    xyz, tri = icosphere_mesh(1)
    M = tri.shape[0]
    s = np.array([0.8, 2.0 + 4.0j])
    pairs = [(a, b) for a in range(0, M, 7) for b in range(M)
             if len(set(tri[a]) & set(tri[b])) == 0][:40]
    ti = np.array([p[0] for p in pairs])
    tj = np.array([p[1] for p in pairs])
    loc = pair_local(xyz, tri, "dnx", s, ti, tj)
    # centroids of 4^5 congruent sub-triangles, barycentric
    subs = [np.eye(3)]
    for _ in range(5):
        nxt = []
        for t in subs:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            nxt += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        subs = nxt
    lam = np.array([t.mean(axis=0) for t in subs])
    for p, (a, b) in enumerate(pairs):
        A, B = xyz[tri[a]], xyz[tri[b]]
        na = np.cross(A[1] - A[0], A[2] - A[0])
        area_a = 0.5 * np.linalg.norm(na)
        na = na / (2 * area_a)
        area_b = 0.5 * np.linalg.norm(np.cross(B[1] - B[0], B[2] - B[0]))
        X, Y = lam @ A, lam @ B
        d = X[:, None, :] - Y[None, :, :]
        r = np.linalg.norm(d, axis=2)
        num = -(d @ na)
        w = area_a * area_b / lam.shape[0] ** 2
        for l, sl in enumerate(s):
            k = num * np.exp(-sl * r) * (1 + sl * r) / (4 * np.pi * r ** 3) * w
            ref = lam.T @ k @ lam
            scale = np.abs(ref).max()
            assert np.abs(loc[p, :, :, l] - ref).max() <= 2e-3 * scale, (a, b, l)


def test_hypersingular_annihilates_constants_at_zero_frequency():
    xyz, tri = lshape_mesh(1)
    g = P1Geometry(xyz, tri)
    nv = g.M
    ii, jj = np.repeat(np.arange(nv), nv), np.tile(np.arange(nv), nv)
    D = p1_galerkin_entries(g, "hyp", np.array([0.0]), ii, jj).reshape(nv, nv)
    assert np.abs(D.sum(axis=1)).max() <= 1e-12 * np.abs(D).sum(axis=1).max()
    assert np.abs(D - D.T).max() <= 1e-6 * np.abs(D).max()   # symmetric up to quadrature


def _sphere_closed_forms(s):
    """Unit sphere, constant density: D1(s) and K'1(s) (values on the surface)."""
    i0 = np.sinh(s) / s
    di0 = (s * np.cosh(s) - np.sinh(s)) / s ** 2
    k0 = np.exp(-s) / s
    dk0 = -np.exp(-s) * (s + 1) / s ** 2
    V1 = (1 - np.exp(-2 * s)) / (2 * s)
    K1 = np.exp(-2 * s) / 2 - V1
    D1 = -s * di0 * (K1 - 0.5) / i0
    Kp1 = 0.5 * (V1 / i0 * s * di0 + V1 / k0 * s * dk0)
    return D1, Kp1


def test_unit_sphere_sums_converge():
    s = np.array([1.0, 2.0 + 1.5j])
    D1, Kp1 = _sphere_closed_forms(s)
    errs = {"hyp": [], "adlp": []}
    for level in (1, 2, 3):
        xyz, tri = icosphere_mesh(level)
        g = P1Geometry(xyz, tri)
        nv = g.M
        ii, jj = np.repeat(np.arange(nv), nv), np.tile(np.arange(nv), nv)
        for op, ref in (("hyp", D1), ("adlp", Kp1)):
            tot = p1_galerkin_entries(g, op, s, ii, jj, n_ss=6).sum(axis=0)
            errs[op].append(np.abs(tot - 4 * np.pi * ref) / np.abs(4 * np.pi * ref))
    for op in errs:
        e = np.array(errs[op])
        ratio = e[:2] / e[1:]
        assert np.all(ratio > 3.0), (op, e, ratio)
        assert np.all(e[2] < 2e-2), (op, e)
