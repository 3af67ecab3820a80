"""Pins for the oracle's compressed operator: error on real blocks and the reordered
product eq. (product) against a plain einsum over the reconstructed dense tensor."""
import numpy as np
import pytest

from inputs import circle_frequencies, cube_mesh, get_config, mesh_for_config, random_rhs
from oracle.hmatrix import Problem, apply, compress_far


@pytest.fixture(scope="module")
def small_problem():
    xyz, tri = cube_mesh(8)
    s = circle_frequencies(16, 10.0, 0.9)
    P = Problem(xyz, tri, s, 16, 1.0)
    eps = 1e-4
    far_res, far_T = [], []
    for blk in P.far:
        res, Tb = compress_far(P, "slp", blk, eps, eps / 100)
        far_res.append(res)
        far_T.append(Tb)
    near_T = [P.block_tensor("slp", blk, False) for blk in P.near]
    return P, eps, far_res, far_T, near_T


def test_small_problem_has_far_and_near(small_problem):
    P, *_ = small_problem
    assert len(P.far) > 50 and len(P.near) > 10


def test_block_errors_within_tolerance(small_problem):
    P, eps, far_res, far_T, _ = small_problem
    num = den = 0.0
    for blk, res, Tb in zip(P.far, far_res, far_T):
        rec = res.reconstruct(blk[1], blk[3], P.L)
        e = np.linalg.norm(rec - Tb)
        num += e * e
        den += np.linalg.norm(Tb) ** 2
        assert e <= 10 * eps * np.linalg.norm(Tb)
    assert np.sqrt(num / den) <= 10 * eps


@pytest.mark.parametrize("mode", ["sum", "per_freq"])
def test_apply_matches_dense_einsum(small_problem, mode):
    P, eps, far_res, far_T, near_T = small_problem
    M, L = P.M, P.L
    C = np.zeros((M, M, L), dtype=complex)
    for blk, res in zip(P.far, far_res):
        rows, cols = P.block_ids(blk)
        C[np.ix_(rows, cols)] = res.reconstruct(blk[1], blk[3], L)
    for blk, Nb in zip(P.near, near_T):
        rows, cols = P.block_ids(blk)
        C[np.ix_(rows, cols)] = Nb
    X = random_rhs(L, M, 3, seed=1)
    Y = apply(P, far_res, near_T, X, mode=mode)
    if mode == "sum":
        ref = np.einsum("ijl,ljb->ib", C, X)
    else:
        ref = np.einsum("ijl,ljb->lib", C, X)
    assert np.linalg.norm(Y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_sum_mode_is_sum_of_per_freq(small_problem):
    P, eps, far_res, far_T, near_T = small_problem
    X = random_rhs(P.L, P.M, 2, seed=2)
    Ys = apply(P, far_res, near_T, X, mode="sum")
    Yp = apply(P, far_res, near_T, X, mode="per_freq")
    assert np.linalg.norm(Ys - Yp.sum(axis=0)) <= 1e-13 * np.linalg.norm(Ys)


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_c2_sampled_blocks_error(kernel):
    cfg = get_config("C2")
    xyz, tri = mesh_for_config("C2")
    s = circle_frequencies(cfg["L"], cfg["c0"], cfg["rho"])
    P = Problem(xyz, tri, s, cfg["leaf"], cfg["eta"])
    rng = np.random.default_rng(11)
    far = np.array(P.far)
    pick = list(rng.choice(len(far), 5, replace=False))
    pick.append(int(np.argmax(far[:, 1] * far[:, 3])))
    for bi in pick:
        blk = tuple(int(v) for v in far[bi])
        res, Tb = compress_far(P, kernel, blk, cfg["eps"], cfg["eps_aca"])
        nt = np.linalg.norm(Tb)
        e = np.linalg.norm(res.reconstruct(blk[1], blk[3], P.L) - Tb)
        assert e <= 10 * cfg["eps"] * nt or (nt == 0 and res.rank == 0)
        assert res.rank < P.L // 2
