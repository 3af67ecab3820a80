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

from oracle.aca3d import aca3d, argmax_tie, face_aca, gram_face


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
