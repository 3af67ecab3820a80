"""Pins of the oracle's P1 double layer collocated at the vertices (eq. bie_semi_diri with
linear continuous trial functions).

* Gauss solid angle: at s = 0 the row sums equal -(1 / 4 pi) times the solid angle that the
  surface subtends at the vertex, evaluated here triangle by triangle by the closed form of
  Van Oosterom and Strackee (1983) for a flat triangle; on the cube that is -1/2, -1/4 and
  -1/8 at face, edge and corner vertices;
* linear functions: sum_j K_ij(s) f(x_j) for f linear equals int_Gamma dG/dn_y f(y) dS_y
  (P1 interpolation is exact), checked against a brute-force midpoint rule on 4^6
  sub-triangles per triangle written here in numpy (independent of the oracle's rules);
* unit sphere: row sums converge to e^{-2s}/2 - (1 - e^{-2s})/(2s) at first order
  (the flat patch around the collocation vertex contributes nothing);
* zero rules: K_ii = 0 exactly (every triangle of the patch holds x_i);
* conjugate frequencies give conjugate entries bitwise;
* every quadrature tier against the collapsed 40 x 40 rule."""
import numpy as np
import pytest

from inputs import circle_frequencies, cube_mesh, icosphere_mesh, lshape_mesh
from oracle.entries import P1Geometry, p1_dlp_entries


def _all_pairs(nv, rows):
    return np.repeat(rows, nv), np.tile(np.arange(nv), rows.shape[0])


def _solid_angle(x, a, b, c):
    """Signed solid angle of the flat triangle (a, b, c) seen from x (Van Oosterom and
    Strackee): tan(Omega / 2) = a . (b x c) / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|)
    with a, b, c relative to x."""
    a, b, c = a - x, b - x, c - x
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = np.dot(a, np.cross(b, c))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * np.arctan2(num, den)


@pytest.mark.parametrize("mesh", ["cube", "lshape"])
def test_p1_gauss_solid_angle(mesh):
    xyz, tri = cube_mesh(4) if mesh == "cube" else lshape_mesh(2)
    g = P1Geometry(xyz, tri)
    nv = g.M
    rows = np.arange(0, nv, 3)
    ii, jj = _all_pairs(nv, rows)
    ref = []
    for i in rows:
        om = sum(_solid_angle(xyz[i], *xyz[t]) for t in tri if i not in t)
        ref.append(om / (4 * np.pi))
    # outward normals: the kernel (x - y) . n_y / (4 pi r^3) integrates to minus the solid angle
    ref = -np.array(ref)
    s = np.array([0.0])
    tiers = p1_dlp_entries(g, s, ii, jj).reshape(rows.shape[0], nv).sum(axis=1).real
    high = p1_dlp_entries(g, s, ii, jj, order=32).reshape(rows.shape[0], nv).sum(axis=1).real
    assert np.abs(tiers - ref).max() < 5e-3, np.abs(tiers - ref).max()
    assert np.abs(high - ref).max() < 2e-4, np.abs(high - ref).max()
    if mesh == "cube":
        # interior solid angles 2 pi (faces), pi (edges), pi / 2 (corners)
        assert set(np.round(ref, 12)) <= {-0.5, -0.25, -0.125}
        assert set(np.round(ref, 12)) == {-0.5, -0.25, -0.125}


def _brute(xyz, tri, x, s, f, levels=6):
    """int_Gamma dG/dn_y(x - y) f(y) dS_y: each triangle not holding x cut into 4^levels
    congruent pieces, kernel times f at each piece's centroid times its area."""
    # barycentric centroids of the 4^levels sub-triangles, built by repeated midpoint split
    subs = [np.eye(3)]
    for _ in range(levels):
        nxt = []
        for t in subs:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            nxt += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        subs = nxt
    lam = np.array([t.mean(axis=0) for t in subs])          # (4^levels, 3)
    total = np.zeros(s.shape[0], dtype=complex)
    for t in tri:
        if np.any(np.all(xyz[t] == x, axis=1)):
            continue
        a, b, c = xyz[t]
        nrm = np.cross(b - a, c - a)
        area = 0.5 * np.linalg.norm(nrm)
        n = nrm / (2 * area)
        y = lam @ xyz[t]
        d = x[None, :] - y
        r = np.linalg.norm(d, axis=1)
        w = area / lam.shape[0] * f(y) * (d @ n) / (4 * np.pi * r ** 3)
        total += (np.exp(-np.outer(s, r)) * (1 + np.outer(s, r))) @ w
    return total


def test_p1_linear_functions_against_brute_force():
    xyz, tri = cube_mesh(2)
    # tilt the cube so that no coordinate plane holds a face (no exact zeros by symmetry)
    th = 0.3
    rot = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    rot = rot @ np.array([[1, 0, 0], [0, np.cos(0.5), -np.sin(0.5)], [0, np.sin(0.5), np.cos(0.5)]])
    xyz = xyz @ rot.T
    g = P1Geometry(xyz, tri)
    nv = g.M
    s = np.array([0.7, 2.0 + 3.0j])
    rows = np.array([0, 5, 11, nv - 1])
    ii, jj = _all_pairs(nv, rows)
    K = p1_dlp_entries(g, s, ii, jj, order=24).reshape(rows.shape[0], nv, -1)
    for f in (lambda y: y[..., 2], lambda y: 1.0 + 2.0 * y[..., 0] - y[..., 1]):
        fv = f(xyz)
        for r, i in enumerate(rows):
            got = (K[r] * fv[:, None]).sum(axis=0)
            ref = _brute(xyz, tri, xyz[i], s, f)
            # scale: the sum of the magnitudes (the value itself vanishes by symmetry at
            # some vertices, e.g. f = z at a face centre)
            scale = (np.abs(K[r]) * np.abs(fv)[:, None]).sum(axis=0).max()
            assert np.abs(got - ref).max() <= 2e-4 * scale, (i, got, ref)


def _sphere_rows(level, s):
    xyz, tri = icosphere_mesh(level)
    g = P1Geometry(xyz, tri)
    nv = g.M
    rows = np.arange(0, nv, max(1, nv // 16))
    ii, jj = _all_pairs(nv, rows)
    return p1_dlp_entries(g, s, ii, jj).reshape(rows.shape[0], nv, -1).sum(axis=1)


def test_p1_unit_sphere_row_sums_converge():
    # first order in h: the flat triangles around the collocation vertex contribute nothing,
    # where the curved surface contributes about -h / 4 (kernel ~ -1 / (8 pi R r) over a
    # disc of radius h on the unit sphere); each refinement halves the error
    s = np.array([1.0, 2.0 + 3.0j, 5.0 - 1.0j])
    exact = np.exp(-2 * s) / 2 - (1 - np.exp(-2 * s)) / (2 * s)
    errs = np.array([np.abs(_sphere_rows(level, s) - exact[None, :]).max(axis=0)
                     for level in (2, 3, 4)])
    ratio = errs[:2] / errs[1:]
    assert np.all((ratio > 1.5) & (ratio < 2.3)), (errs, ratio)
    assert np.all(errs[2] < 0.03), errs


def test_p1_zero_diagonal_and_conjugate_symmetry():
    xyz, tri = icosphere_mesh(2)
    g = P1Geometry(xyz, tri)
    nv = g.M
    d = np.arange(nv)
    s = circle_frequencies(8, 10.0, 0.9)
    K = p1_dlp_entries(g, s, d, d)
    assert np.all(K == 0)
    rng = np.random.default_rng(3)
    ii, jj = rng.integers(0, nv, 500), rng.integers(0, nv, 500)
    E = p1_dlp_entries(g, s, ii, jj)
    assert np.array_equal(E[:, ::-1], np.conj(E))


def test_p1_tiers_converge_to_high_order():
    xyz, tri = icosphere_mesh(3)
    g = P1Geometry(xyz, tri)
    nv = g.M
    s = circle_frequencies(8, 20.0, 0.95)
    rng = np.random.default_rng(7)
    ii = rng.integers(0, nv, 3000)
    jj = rng.integers(0, nv, 3000)
    # neighbours (close pairs: the collapsed tiers) as well as random (mostly 6-point) pairs
    nb = g.tri[g.ptri[g.pptr[ii[:1000]]]]
    jj[:1000] = nb[np.arange(1000), rng.integers(0, 3, 1000)]
    far = np.zeros(ii.shape[0], dtype=np.int32)
    E = p1_dlp_entries(g, s, ii, jj, far)
    ref = p1_dlp_entries(g, s, ii, jj, order=40)
    scale = np.abs(ref).max(axis=1)
    ok = scale > 0
    rel = np.abs(E - ref).max(axis=1)[ok] / scale[ok]
    assert rel.max() < 1e-3, rel.max()
    assert np.median(rel) < 1e-5


def test_p1_problem_partition_and_compression():
    """Vertex tree: every (vertex, vertex) pair covered exactly once; admissible pairs have
    separated support boxes; far blocks of the P1 double layer compress by Algorithm 1 to
    within 10 eps."""
    from oracle.aca3d import aca3d
    from oracle.hmatrix import Problem
    xyz, tri = cube_mesh(8)
    s = circle_frequencies(16, 10.0, 0.9)
    op = Problem(xyz, tri, s, 16, 1.0, scheme="p1")
    nv = xyz.shape[0]
    assert op.M == nv and np.array_equal(np.sort(op.perm), np.arange(nv))
    cover = np.zeros((nv, nv), dtype=np.int32)
    for r0, m, c0, n in op.far + op.near:
        cover[r0:r0 + m, c0:c0 + n] += 1
    assert np.all(cover == 1)
    assert len(op.far) >= 40
    rng = np.random.default_rng(2)
    for b in rng.choice(len(op.far), 12, replace=False):
        blk = op.far[b]
        T = op.block_tensor("dlp", blk, True)
        res = aca3d(T, 1e-4, 1e-6)
        C = res.reconstruct(blk[1], blk[3], op.L)
        assert np.linalg.norm(C - T) <= 10 * 1e-4 * np.linalg.norm(T), (blk, res.rank)
