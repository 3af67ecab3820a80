"""P1 double layer collocated at the vertices (scheme "p1"; Sec. 3, eq. bie_semi_diri with
linear continuous trial functions) on the GPU against the oracle.

Bars: entries (the test hook, far and near rules) within 1e-12 of the oracle's entry
magnitude; every near block of the 386-vertex cube within 1e-12 of ||T||_F; far blocks
whose crosses pick the oracle's pivots and ranks within 1e-6 of ||T||_F of the oracle's
reconstruction (at least 90 % of the blocks), every block within 10 eps of T; the apply
(complex128, both modes) within 1e-12 of the oracle's eq. (product) over the exported
operator; on the 10242-vertex sphere sampled far blocks within 10 eps of the oracle's T."""
import numpy as np
import pytest

from gpu_common import context, gpu_problem, log, oracle_problem, reconstruct, rel_fro

pytestmark = pytest.mark.gpu


class _Cross:
    def __init__(self, c):
        self.U, self.W, self.f = c["U"], c["W"], c["f"]


class _Block:
    def __init__(self, e):
        self.crosses = [_Cross(c) for c in e["crosses"]]


def test_p1_entries_vs_oracle():
    from oracle.entries import P1Geometry, p1_dlp_entries
    cfg, prob, (xyz, tri, s) = gpu_problem("p1cube386")
    g = P1Geometry(xyz, tri)
    nv = xyz.shape[0]
    rng = np.random.default_rng(11)
    n = 4000
    ii = rng.integers(0, nv, n)
    jj = rng.integers(0, nv, n)
    # neighbours and diagonal entries (zero rule, collapsed tiers)
    nb = g.tri[g.ptri[g.pptr[ii[:1500]]]]
    jj[:1500] = nb[np.arange(1500), rng.integers(0, 3, 1500)]
    jj[1500:1600] = ii[1500:1600]
    far = (rng.random(n) < 0.3).astype(np.int32)
    far[:1600] = 0
    ks = rng.integers(0, len(s), n)
    got = prob.eval_entries("dlp", ii, jj, ks, far)
    ref = p1_dlp_entries(g, s, ii, jj, far)[np.arange(n), ks]
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    log(f"P1 entries vs oracle: {n} entries, max |diff| / max |entry| = {err:.2e}")
    assert np.all(got[1500:1600] == 0)
    assert err <= 1e-12


def test_p1_build_vs_oracle():
    from oracle.aca3d import aca3d
    cfg, prob, _ = gpu_problem("p1cube386")
    _, op = oracle_problem("p1cube386")
    h = prob.build("dlp")
    far, near = prob.blocks()
    assert far.shape[0] == len(op.far) and near.shape[0] == len(op.near)
    worst_near = 0.0
    for b in range(near.shape[0]):
        blk = tuple(int(v) for v in near[b])
        T = op.block_tensor("dlp", blk, False)
        N = np.transpose(h.near_block(b, blk[1], blk[3]), (0, 2, 1))
        nt = np.linalg.norm(T)
        e = np.linalg.norm(N - T) / nt if nt > 0 else np.abs(N).max()
        worst_near = max(worst_near, e)
    assert worst_near <= 1e-12, worst_near
    n_same = 0
    worst_par = worst_err = 0.0
    for b in range(far.shape[0]):
        blk = tuple(int(v) for v in far[b])
        T = op.block_tensor("dlp", blk, True)
        nt = np.linalg.norm(T)
        C = reconstruct(h, b)
        err = np.linalg.norm(C - T) / nt
        worst_err = max(worst_err, err)
        assert err <= 10 * cfg["eps"], (b, blk, err)
        o = aca3d(T, cfg["eps"], cfg["eps_aca"])
        e = h.export_block(b)
        same = e["rank"] == o.rank and all(
            c["k"] == oc.k and c["i"] == oc.i and c["j"] == oc.j and c["rho"] == oc.U.shape[1]
            for c, oc in zip(e["crosses"], o.crosses))
        if same:
            n_same += 1
            par = np.linalg.norm(C - o.reconstruct(blk[1], blk[3], op.L)) / nt
            worst_par = max(worst_par, par)
            assert par <= 1e-6, (b, blk, par)
    st = h.stats()
    log(f"P1 cube 386 vertices: {far.shape[0]} far blocks, same pivots {n_same}, worst parity "
        f"{worst_par:.2e}, worst error {worst_err:.2e}; near worst {worst_near:.2e}; ranks "
        f"{st['rank_min']}..{st['rank_max']} mean {st['rank_mean']:.2f}, compression {st['compression']:.3f}")
    assert n_same >= 0.9 * far.shape[0]


@pytest.mark.parametrize("mode,nrhs", [("sum", 1), ("sum", 3), ("per_freq", 2)])
def test_p1_apply_vs_oracle(mode, nrhs):
    import torch
    from inputs import random_rhs
    from oracle.hmatrix import apply as oapply
    cfg, prob, (xyz, tri, s) = gpu_problem("p1cube386")
    _, op = oracle_problem("p1cube386")
    h = prob.build("dlp")
    far, near = prob.blocks()
    fres = [_Block(h.export_block(b)) for b in range(far.shape[0])]
    ntens = [np.transpose(h.near_block(b, int(near[b, 1]), int(near[b, 3])), (0, 2, 1))
             for b in range(near.shape[0])]
    X = random_rhs(len(s), xyz.shape[0], nrhs, seed=90 + nrhs)
    Y = h.apply(torch.from_numpy(X).cuda(), mode=mode)
    torch.cuda.synchronize()
    Y = Y.cpu().numpy()
    Yo = oapply(op, fres, ntens, X, mode=mode)
    e = rel_fro(Y, Yo)
    log(f"P1 apply {mode} {nrhs} rhs vs oracle product: {e:.2e}")
    assert e <= 1e-12


def test_p1_rejects_other_kernels_and_mixed():
    import paper_2312_11219_amd as gaca
    from paper_2312_11219_amd._binding import GacaError
    cfg, prob, (xyz, tri, s) = gpu_problem("p1cube386")
    with pytest.raises(GacaError, match="UNSUPPORTED"):
        prob.build("slp")
    with pytest.raises(GacaError, match="UNSUPPORTED"):
        prob.build_both()
    with pytest.raises(GacaError, match="UNSUPPORTED"):
        gaca.Problem(context(), xyz, tri, s, scheme="p1", precision="mixed")


def test_p1_sphere_10242_sampled_blocks():
    """The P1 double layer at the 20480-triangle sphere's size (10242 vertices, L = 128):
    seeded sampled far blocks (and the largest) within 10 eps of the oracle's T, sampled near
    blocks within 1e-12."""
    from oracle.hmatrix import Problem
    cfg, prob, (xyz, tri, s) = gpu_problem("P1")
    h = prob.build("dlp")
    st = h.stats()
    far, near = prob.blocks()
    op = Problem(xyz, tri, s, cfg["leaf"], cfg["eta"], scheme="p1")
    rng = np.random.default_rng(21)
    side = np.maximum(far[:, 1], far[:, 3])
    pick = sorted(set(rng.choice(np.nonzero(side <= 256)[0], 6, replace=False).tolist()
                      + [int(np.argmax(far[:, 1] * far[:, 3]))]))
    worst = 0.0
    for b in pick:
        blk = tuple(int(v) for v in far[b])
        T = op.block_tensor("dlp", blk, True)
        err = rel_fro(reconstruct(h, b), T)
        worst = max(worst, err)
        assert err <= 10 * cfg["eps"], (b, blk, err)
    wn = 0.0
    for b in rng.choice(near.shape[0], 12, replace=False):
        blk = tuple(int(v) for v in near[b])
        T = op.block_tensor("dlp", blk, False)
        N = np.transpose(h.near_block(int(b), blk[1], blk[3]), (0, 2, 1))
        wn = max(wn, rel_fro(N, T) if np.linalg.norm(T) > 0 else np.abs(N).max())
    log(f"P1 sphere 10242 vertices L {len(s)}: build {st['ms_total']:.1f} ms (near {st['ms_near']:.1f}, "
        f"far {st['ms_far']:.1f}), {far.shape[0]} far / {near.shape[0]} near blocks, ranks mean "
        f"{st['rank_mean']:.2f} max {st['rank_max']}, compression {st['compression']:.4f}; sampled far "
        f"worst {worst:.2e}, near worst {wn:.2e}")
    assert wn <= 1e-12
