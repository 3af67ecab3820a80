"""Pins for the oracle's 3D-ACA (Algorithm 1) and face ACA.

* exact recovery of random complex tensors of known 3-D rank and face rank;
* eps = 0 with exact faces reproduces any tensor after L crosses;
* exact faces: f_l[k_l] = 1 and f_l[k_p] = 0 for earlier crosses (fibre interpolation);
* the recursion eq. (norm) equals the directly computed norm of C^(l);
* lowest-index tie rule; zero block -> rank 0 after three zero faces;
* face ACA recovers random rank-rho matrices exactly and approximates smooth-kernel blocks
  within a constant times eps_aca with a rank close to the truncated SVD rank.
"""
import numpy as np
import pytest

from oracle.aca3d import (aca3d, aca3d_dense, argmax_tie, face_aca, gram_face, index_pivot,
                          near_storage_compressed, recompress)


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _known_rank_tensor(rng, m, n, L, R, rho):
    T = np.zeros((m, n, L), dtype=complex)
    for _ in range(R):
        H = _crandn(rng, m, rho) @ _crandn(rng, rho, n)
        T += H[:, :, None] * _crandn(rng, L)[None, None, :]
    return T


@pytest.mark.parametrize("R,rho", [(1, 1), (2, 3), (4, 2), (8, 3)])
def test_known_rank_recovered(R, rho):
    rng = np.random.default_rng(10 + R)
    m, n, L = 20, 17, 12
    T = _known_rank_tensor(rng, m, n, L, R, rho)
    res = aca3d(T, 1e-10, 1e-12)
    assert res.rank == R
    err = np.linalg.norm(res.reconstruct(m, n, L) - T) / np.linalg.norm(T)
    assert err < 1e-12


def test_eps_zero_reproduces_tensor():
    rng = np.random.default_rng(2)
    m, n, L = 6, 5, 4
    T = _crandn(rng, m, n, L)
    res = aca3d(T, 0.0, 0.0)
    assert res.rank == L
    err = np.linalg.norm(res.reconstruct(m, n, L) - T) / np.linalg.norm(T)
    assert err < 1e-12


def test_fibre_interpolation_properties():
    rng = np.random.default_rng(3)
    m, n, L = 7, 6, 9
    T = _crandn(rng, m, n, L)
    res = aca3d(T, 0.0, 0.0, max_rank3d=5)
    ks = [c.k for c in res.crosses]
    assert len(set(ks)) == len(ks)
    for l, c in enumerate(res.crosses):
        assert abs(c.f[c.k] - 1.0) < 1e-12
        for p in range(l):
            assert abs(c.f[res.crosses[p].k]) < 1e-12
        # the 3-D cross reproduces the face and the fibre through the pivot
    C = res.reconstruct(m, n, L)
    for c in res.crosses:
        assert np.allclose(C[:, :, c.k], T[:, :, c.k], atol=1e-12)
        assert np.allclose(C[c.i, c.j, :], T[c.i, c.j, :], atol=1e-12)


def test_norm_recursion_equals_direct():
    rng = np.random.default_rng(4)
    m, n, L = 15, 12, 10
    T = _known_rank_tensor(rng, m, n, L, 6, 4) + 1e-3 * _crandn(rng, m, n, L)
    res = aca3d(T, 1e-8, 1e-10)
    C = res.reconstruct(m, n, L)
    assert abs(np.sqrt(res.norm2) - np.linalg.norm(C)) < 1e-12 * np.linalg.norm(C)
    # Gram cache
    for a, ca in enumerate(res.crosses):
        for b, cb in enumerate(res.crosses):
            direct = np.vdot((cb.U @ cb.W.T), (ca.U @ ca.W.T))
            assert abs(res.gram[a][b] - direct) < 1e-10 * abs(res.gram[a][a])


def test_argmax_tie_lowest_index():
    a = np.array([1.0, 3.0, 3.0 * (1 - 1e-12), 2.0, 3.0])
    assert argmax_tie(a) == 1
    assert argmax_tie(a, np.array([True, False, True, True, True])) == 2
    b = np.array([1.0, 3.0, 3.0 * (1 - 1e-6)])
    assert argmax_tie(b[::-1]) == 1


def test_zero_block():
    T = np.zeros((5, 4, 6), dtype=complex)
    res = aca3d(T, 1e-6, 1e-8)
    assert res.rank == 0 and res.zero_faces == 3
    assert list(np.nonzero(res.used)[0]) == [0, 1, 2]


def test_first_frequency_is_zero_and_next_is_unused_argmax():
    rng = np.random.default_rng(5)
    T = _crandn(rng, 6, 6, 8)
    res = aca3d(T, 0.0, 0.0, max_rank3d=3)
    assert res.crosses[0].k == 0
    f = res.crosses[0].f
    a2 = np.abs(f) ** 2
    a2[0] = -1
    assert res.crosses[1].k == int(np.argmax(a2))


@pytest.mark.parametrize("rho", [1, 3, 8])
def test_face_aca_exact_low_rank(rho):
    rng = np.random.default_rng(20 + rho)
    A = _crandn(rng, 30, rho) @ _crandn(rng, rho, 25)
    U, W = face_aca(A, 1e-14, 0.0, 25)
    assert U.shape[1] <= rho + 1
    assert np.linalg.norm(U @ W.T - A) < 1e-12 * np.linalg.norm(A)


def test_face_aca_zero_rows():
    """Zero rows (rows 0, 3 and 7 exactly zero) and a residual that turns zero while rows of a
    second, decoupled block remain: R = [[A, 0], [0, B]] with A (rows 0-7, columns 0-5) of
    rank 2 and B (rows 8-15, columns 6-11) of rank 3.  The search starts at row 0 (zero, so
    row 1 is next in index order); once A is exhausted every unused row of A has a zero
    residual and is passed over in index order, so the first cross in B is at row 8; the
    face is recovered exactly with 5 crosses."""
    rng = np.random.default_rng(11)
    cplx = lambda *sh: rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    R = np.zeros((16, 12), complex)
    A = cplx(8, 2) @ cplx(2, 6)
    A[[0, 3, 7]] = 0.0
    R[:8, :6] = A
    R[8:, 6:] = cplx(8, 3) @ cplx(3, 6)
    U, W, piv = face_aca(R, 1e-14, 1e-10 * np.abs(R).max(), 16, return_pivots=True)
    rows = [p[0] for p in piv]
    assert U.shape[1] == 5 and len(rows) == 5
    assert rows[0] == 1 and rows[2] == 8
    assert not {0, 3, 7} & set(rows)
    assert set(rows[:2]) <= {1, 2, 4, 5, 6} and set(rows[2:]) <= set(range(8, 16))
    assert np.linalg.norm(U @ W.T - R) <= 1e-12 * np.linalg.norm(R)


def test_face_aca_smooth_kernel_vs_svd():
    # two separated point clouds, Laplace-domain kernel at one frequency
    rng = np.random.default_rng(6)
    x = rng.random((60, 3))
    y = rng.random((50, 3)) + np.array([2.5, 0, 0])
    r = np.linalg.norm(x[:, None, :] - y[None, :, :], axis=2)
    s = 3.0 + 4.0j
    A = np.exp(-s * r) / (4 * np.pi * r)
    for eps in (1e-4, 1e-6, 1e-8):
        U, W = face_aca(A, eps, 0.0, 50)
        err = np.linalg.norm(U @ W.T - A) / np.linalg.norm(A)
        sv = np.linalg.svd(A, compute_uv=False)
        tail = np.sqrt(np.cumsum((sv ** 2)[::-1]))[::-1] / np.linalg.norm(sv)
        svd_rank = int(np.argmax(tail <= eps))
        assert err < 30 * eps
        assert U.shape[1] <= 2 * svd_rank + 2


def test_gram_face():
    rng = np.random.default_rng(7)
    Ua, Wa, Ub, Wb = _crandn(rng, 5, 2), _crandn(rng, 4, 2), _crandn(rng, 5, 3), _crandn(rng, 4, 3)
    Ha, Hb = Ua @ Wa.T, Ub @ Wb.T
    assert abs(gram_face(Ua, Wa, Ub, Wb) - np.sum(Ha * Hb.conj())) < 1e-12


def _lowrank_face(rng, m, n, rho, decay):
    U = (rng.standard_normal((m, rho)) + 1j * rng.standard_normal((m, rho))) * decay[None, :]
    W = rng.standard_normal((n, rho)) + 1j * rng.standard_normal((n, rho))
    return U, W


@pytest.mark.parametrize("m,n,rho", [(40, 30, 12), (25, 60, 20), (7, 9, 7)])
def test_recompress_is_truncated_svd(m, n, rho):
    """QR of both factors + SVD of the small core = the SVD of the dense face: the singular
    values of U W^T (numpy SVD of the m x n matrix), the kept rank is the smallest whose
    discarded tail is within eps of the norm, and U' W'^T is the truncated SVD (Eckart-Young)."""
    rng = np.random.default_rng(m + n + rho)
    U, W = _lowrank_face(rng, m, n, rho, np.logspace(0, -9, rho))
    H = U @ W.T
    Ud, sd, Vh = np.linalg.svd(H)
    for eps in (1e-3, 1e-6, 0.0):
        U2, W2, sig = recompress(U, W, eps)
        r = len(sig)
        assert np.allclose(sig, sd[:r], rtol=1e-9, atol=1e-12 * sd[0])
        tails = np.sqrt(np.cumsum((sd[:rho] ** 2)[::-1])[::-1])
        want = max(1, int(np.sum(tails > eps * np.linalg.norm(H))))
        assert r == want, (eps, r, want)
        Ht = (Ud[:, :r] * sd[:r]) @ Vh[:r]
        assert np.linalg.norm(U2 @ W2.T - Ht) <= 1e-9 * np.linalg.norm(H)
        assert np.linalg.norm(U2 @ W2.T - H) <= max(eps, 1e-12) * np.linalg.norm(H) * (1 + 1e-9)


def test_recompress_reference_norm():
    """The truncation tolerance is relative to the operator face (ref2 + ||H||^2): a face that
    is small against the part already represented is truncated further."""
    rng = np.random.default_rng(3)
    U, W = _lowrank_face(rng, 30, 30, 10, np.logspace(0, -6, 10))
    nh2 = np.linalg.norm(U @ W.T) ** 2
    r0 = len(recompress(U, W, 1e-4)[2])
    r1 = len(recompress(U, W, 1e-4, ref2=1e4 * nh2)[2])
    assert r1 < r0


def test_index_pivot_rank_one_is_exact():
    """eq. (index) on a rank-1 face picks the true largest entry."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        u = rng.standard_normal(17) + 1j * rng.standard_normal(17)
        w = rng.standard_normal(23) + 1j * rng.standard_normal(23)
        U2, W2, sig = recompress(u[:, None], w[:, None], 1e-8)
        i, j = index_pivot(U2, W2, sig)
        H = np.outer(u, w)
        assert (i, j) == np.unravel_index(np.argmax(np.abs(H)), H.shape)


@pytest.mark.parametrize("pivot", ["dense", "index"])
def test_aca3d_recompressed_on_kernel_block(pivot):
    """The 3D-ACA with recompressed faces (both pivot rules) on a single layer block of the
    768-triangle cube: error within 10 eps and less face storage than without."""
    from inputs import circle_frequencies, cube_mesh
    from oracle.hmatrix import Problem
    xyz, tri = cube_mesh(8)
    s = circle_frequencies(16, 10.0, 0.9)
    op = Problem(xyz, tri, s, 16, 1.0)
    sizes = [b[1] * b[3] for b in op.far]
    blk = op.far[int(np.argmax(sizes))]
    T = op.block_tensor("slp", blk, True)
    eps = 1e-4
    plain = aca3d(T, eps, eps / 100)
    rec = aca3d(T, eps, eps / 100, recompress_faces=True, pivot=pivot)
    m, n, L = T.shape
    err = np.linalg.norm(rec.reconstruct(m, n, L) - T) / np.linalg.norm(T)
    st_plain = sum(c.U.shape[1] * (m + n) for c in plain.crosses)
    st_rec = sum(c.U.shape[1] * (m + n) for c in rec.crosses)
    assert err <= 10 * eps
    assert st_rec < st_plain


@pytest.mark.parametrize("R", [1, 3, 6])
def test_dense_faces_known_frequency_rank(R):
    """T = sum_{p<R} A_p (x) g_p with dense full-rank A_p: the dense-face 3D-ACA stops with R
    crosses and reproduces T to roundoff; its recursive norm equals ||T||^2."""
    rng = np.random.default_rng(R + 40)
    m, n, L = 12, 9, 20
    T = np.zeros((m, n, L), complex)
    for _ in range(R):
        A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
        g = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        T += A[:, :, None] * g[None, None, :]
    res = aca3d_dense(T, 1e-10)
    assert res.rank == R
    C = res.reconstruct(m, n, L)
    assert np.linalg.norm(C - T) <= 1e-12 * np.linalg.norm(T)
    assert abs(res.norm2 - np.linalg.norm(C) ** 2) <= 1e-10 * np.linalg.norm(C) ** 2
    # fibre interpolation: f_l[k_l] = 1 and f_l[k_p] = 0 for p < l (dense faces are exact)
    for l, c in enumerate(res.crosses):
        assert abs(c.f[c.k] - 1.0) < 1e-12
        for p in range(l):
            assert abs(c.f[res.crosses[p].k]) < 1e-10


def test_dense_faces_eps_zero_and_zero_block():
    rng = np.random.default_rng(7)
    T = rng.standard_normal((5, 4, 6)) + 1j * rng.standard_normal((5, 4, 6))
    res = aca3d_dense(T, 0.0)
    assert res.rank == 6
    assert np.linalg.norm(res.reconstruct(5, 4, 6) - T) <= 1e-12 * np.linalg.norm(T)
    Z = aca3d_dense(np.zeros((5, 4, 6), complex), 1e-6)
    assert Z.rank == 0 and Z.zero_faces == 3


def test_dense_faces_kernel_block_and_storage_rule():
    """A near block of the 3072-triangle cube's single layer (self and neighbour entries):
    error within 10 eps of the dense block; the storage rule keeps it compressed only when
    rank (m n + L) < m n L."""
    from inputs import circle_frequencies, cube_mesh
    from oracle.hmatrix import Problem
    xyz, tri = cube_mesh(16)
    s = circle_frequencies(64, 20.0, 0.95)
    op = Problem(xyz, tri, s, 32, 1.0)
    blk = op.near[0]
    T = op.block_tensor("slp", blk, False)
    eps = 1e-6
    res = aca3d_dense(T, eps)
    m, n, L = T.shape
    assert np.linalg.norm(res.reconstruct(m, n, L) - T) <= 10 * eps * np.linalg.norm(T)
    assert near_storage_compressed(m, n, L, res.rank, res.capped) == (res.rank * (m * n + L) < m * n * L)
    assert not near_storage_compressed(m, n, L, L, False)
    assert not near_storage_compressed(m, n, L, 2, True)
