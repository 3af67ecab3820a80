"""Near-field 3D-ACA with dense faces (option near_aca; Sec. 4 remarks on the non-admissible
blocks and the "No Lwr" variant of Sec. 5) against the oracle's aca3d_dense on the same
blocks, and the apply of the compressed operator against the oracle's eq. (product) over the
exported blocks.

Bars: per near block, the library stores it compressed exactly when the oracle's storage rule
does and with the oracle's rank for at least 95% of the blocks (the rest differ by a tie of
the pivot search); where the ranks agree, the expanded block within 1e-10 of ||T||_F of the
oracle's reconstruction; every block within 10 eps of T (FP64) or 10 eps + 1e-5 (mixed).
Apply (VALU kernels, complex128): within 1e-12 relative Frobenius of the oracle's product over
the exported operator, and within 10 eps of the apply of the same operator with dense near
blocks."""
import numpy as np
import pytest

from gpu_common import gpu_problem, log, oracle_problem, rel_fro

pytestmark = pytest.mark.gpu


class _Cross:
    def __init__(self, c):
        self.U, self.W, self.f = c["U"], c["W"], c["f"]


class _Block:
    def __init__(self, e):
        self.crosses = [_Cross(c) for c in e["crosses"]]


def _near_vs_oracle(name, kernel, precision):
    from oracle.aca3d import aca3d_dense, near_storage_compressed
    cfg, prob, (_, _, s) = gpu_problem(name, near_aca=1, precision=precision)
    _, op = oracle_problem(name)
    h = prob.build(kernel)
    _, near = prob.blocks()
    ranks = h.near_ranks()
    L = len(s)
    assert ranks.shape[0] == near.shape[0]
    n_same = n_comp_o = 0
    worst_par = worst_err = 0.0
    tol = 10 * cfg["eps"] + (1e-5 if precision == "mixed" else 0.0)
    for b in range(near.shape[0]):
        blk = tuple(int(v) for v in near[b])
        m, n = blk[1], blk[3]
        T = op.block_tensor(kernel, blk, False)                 # m x n x L
        nt = np.linalg.norm(T)
        o = aca3d_dense(T, cfg["eps"], max_rank3d=min(L, 64))
        comp_o = m * n <= 1024 and near_storage_compressed(m, n, L, o.rank, o.capped)
        n_comp_o += comp_o
        Nb = np.transpose(h.near_block(b, m, n), (0, 2, 1))     # m x n x L
        if nt == 0:   # e.g. double layer between coplanar clusters
            assert np.abs(Nb).max() == 0
            n_same += int(ranks[b]) == o.rank == 0
            continue
        err = np.linalg.norm(Nb - T) / nt
        worst_err = max(worst_err, err)
        assert err <= tol, (b, blk, err, int(ranks[b]))
        if precision != "fp64":
            continue
        same = (ranks[b] >= 0) == comp_o and (not comp_o or int(ranks[b]) == o.rank)
        if same:
            n_same += 1
            ref = o.reconstruct(m, n, L) if comp_o else T
            par = np.linalg.norm(Nb - ref) / nt
            worst_par = max(worst_par, par)
            assert par <= 1e-10, (b, blk, par)
    st = h.stats()
    log(f"near_aca {name} {kernel} {precision}: {near.shape[0]} near blocks, "
        f"{st['n_near_compressed']} compressed (oracle {n_comp_o}), ranks mean "
        f"{st['near_rank_mean']:.2f} max {st['near_rank_max']}, same as oracle {n_same}, "
        f"worst parity {worst_par:.2e}, worst error {worst_err:.2e}, near bytes "
        f"{st['bytes_near'] / 1e6:.2f} MB, {st['ms_near_aca']:.1f} ms")
    assert st["n_near_compressed"] == int((ranks >= 0).sum()) and st["n_near_compressed"] > 0
    if precision == "fp64":
        assert n_same >= 0.95 * near.shape[0]
    return prob, h, st


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_near_aca_cube768_vs_oracle(kernel):
    _near_vs_oracle("cube768", kernel, "fp64")


def test_near_aca_cube768_mixed():
    _, h, st = _near_vs_oracle("cube768", "slp", "mixed")
    _, plain, _ = gpu_problem("cube768", precision="mixed")
    sp = plain.build("slp").stats()
    assert st["bytes_near"] < sp["bytes_near"]


def test_near_aca_galerkin_lshape768():
    _near_vs_oracle("lshape768", "slp", "fp64")


@pytest.mark.parametrize("mode,nrhs", [("sum", 1), ("sum", 3), ("sum", 6), ("per_freq", 2)])
def test_near_aca_apply_vs_oracle(mode, nrhs):
    import torch
    from inputs import random_rhs
    from oracle.hmatrix import apply as oapply
    cfg, prob, (_, tri, s) = gpu_problem("cube768", near_aca=1)
    _, op = oracle_problem("cube768")
    h = prob.build("slp")
    far, near = prob.blocks()
    fres = [_Block(h.export_block(b)) for b in range(far.shape[0])]
    ntens = [np.transpose(h.near_block(b, int(near[b, 1]), int(near[b, 3])), (0, 2, 1))
             for b in range(near.shape[0])]
    X = random_rhs(len(s), tri.shape[0], nrhs, seed=70 + nrhs)
    Xd = torch.from_numpy(X).cuda()
    Y = h.apply(Xd, mode=mode)
    Y2 = h.apply(Xd, mode=mode)      # the workspace is reused
    _, plain, _ = gpu_problem("cube768")
    Yp = plain.build("slp").apply(Xd, mode=mode)
    torch.cuda.synchronize()
    Y, Y2, Yp = Y.cpu().numpy(), Y2.cpu().numpy(), Yp.cpu().numpy()
    Yo = oapply(op, fres, ntens, X, mode=mode)
    e_or, e_pl = rel_fro(Y, Yo), rel_fro(Y, Yp)
    log(f"near_aca apply {mode} {nrhs} rhs: vs oracle product {e_or:.2e}, vs dense-near apply {e_pl:.2e}")
    assert np.array_equal(Y, Y2)
    assert e_or <= 1e-12
    assert e_pl <= 10 * cfg["eps"]


def test_near_aca_noalloc_unsupported():
    import torch
    from paper_2312_11219_amd._binding import GacaError
    _, prob, (_, tri, s) = gpu_problem("cube768", near_aca=1)
    h = prob.build("slp")
    X = torch.zeros((len(s), tri.shape[0], 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(GacaError, match="UNSUPPORTED"):
        h.apply(X, noalloc=True)
