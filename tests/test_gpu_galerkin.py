"""GPU parity of the Galerkin P0 single layer (near field classes, far 6 x 6 rule, 3D-ACA)
against the FP64 oracle, through the C ABI.  Same bars as the collocation tests."""
import numpy as np
import pytest

from gpu_common import gpu_problem, log, oracle_problem, reconstruct, rel_fro, workload

pytestmark = pytest.mark.gpu


def test_galerkin_eval_entries_all_classes():
    from oracle.entries import Geometry
    from oracle.galerkin import galerkin_entries
    cfg, prob, (xyz, tri, s) = gpu_problem("lshape768")
    M, L = tri.shape[0], s.shape[0]
    rng = np.random.default_rng(8)
    n = 3000
    i = rng.integers(0, M, n)
    j = rng.integers(0, M, n)
    j[:100] = i[:100]
    cen = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3
    for t in range(100, 900):
        d = np.linalg.norm(cen - cen[i[t]], axis=1)
        j[t] = int(np.argsort(d)[1 + t % 10])
    k = rng.integers(0, L, n)
    far = (rng.random(n) < 0.3).astype(np.int32)
    far[:900] = 0
    got = prob.eval_entries("slp", i, j, k, far)
    ref_all, tier = galerkin_entries(Geometry(xyz, tri), "slp", s, i, j, far, return_tier=True)
    assert set(np.unique(tier)) == {0, 1, 2, 3, 4, 5}
    ref = ref_all[np.arange(n), k]
    scale = np.abs(ref_all).max(axis=1)
    err = np.abs(got - ref) / scale
    log("galerkin entries max rel err", err.max(), "by class",
        [float(err[tier == c].max()) for c in range(6)])
    assert err.max() < 1e-12


def test_galerkin_near_blocks():
    cfg, prob, _ = gpu_problem("lshape768")
    ocfg, op = oracle_problem("lshape768")
    h = prob.build("slp")
    far, near = prob.blocks()
    worst = 0.0
    for b in range(0, near.shape[0], 5):
        blk = tuple(int(v) for v in near[b])
        got = h.near_block(b, blk[1], blk[3])
        ref = np.transpose(op.block_tensor("slp", blk, False), (0, 2, 1))
        worst = max(worst, rel_fro(got, ref))
    log("galerkin near worst", worst)
    assert worst < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_galerkin_far_aca(precision):
    from oracle.aca3d import aca3d
    cfg, prob, _ = gpu_problem("lshape768", precision=precision)
    ocfg, op = oracle_problem("lshape768")
    h = prob.build("slp")
    far, _ = prob.blocks()
    same = 0
    pnum = enum = den = 0.0
    for b in range(far.shape[0]):
        blk = tuple(int(v) for v in far[b])
        T = op.block_tensor("slp", blk, True)
        o = aca3d(T, cfg["eps"], cfg["eps_aca"])
        C = reconstruct(h, b)
        Co = o.reconstruct(blk[1], blk[3], op.L)
        e = h.export_block(b)
        same += e["rank"] == o.rank and all(c["k"] == oc.k and c["i"] == oc.i and c["j"] == oc.j
                                            for c, oc in zip(e["crosses"], o.crosses))
        pnum += np.linalg.norm(C - Co) ** 2
        enum += np.linalg.norm(C - T) ** 2
        den += np.linalg.norm(T) ** 2
    par, err = np.sqrt(pnum / den), np.sqrt(enum / den)
    log(f"galerkin {precision}: blocks {far.shape[0]} same pivots {same} parity {par:.3e} err {err:.3e}")
    if precision == "fp64":
        assert par < 1e-6 and same >= 0.95 * far.shape[0]
    assert err < 10 * cfg["eps"] + (1e-5 if precision == "mixed" else 0.0)


def test_c4_sampled_blocks():
    from oracle.aca3d import aca3d
    cfg, prob, _ = gpu_problem("C4")
    ocfg, op = oracle_problem("C4")
    h = prob.build("slp")
    far, near = prob.blocks()
    st = h.stats()
    log("C4 stats", {k: v for k, v in st.items() if k.startswith(("n_", "rank", "ms", "compression"))})
    rng = np.random.default_rng(31)
    sizes = far[:, 1] * far[:, 3]
    cand = np.nonzero(sizes <= 96 * 96)[0]
    big = np.nonzero(np.minimum(far[:, 1], far[:, 3]) >= 256)[0]
    assert big.size >= 2
    pick = sorted(rng.choice(cand, 8, replace=False).tolist() + rng.choice(big, 2, replace=False).tolist())
    num = den = pnum = 0.0
    for b in pick:
        blk = tuple(int(v) for v in far[b])
        T = op.block_tensor("slp", blk, True)
        o = aca3d(T, cfg["eps"], cfg["eps_aca"])
        C = reconstruct(h, b)
        nb = np.linalg.norm(C - o.reconstruct(blk[1], blk[3], op.L)) ** 2
        pnum += nb
        num += np.linalg.norm(C - T) ** 2
        den += np.linalg.norm(T) ** 2
        log(f"C4 block {b} {blk[1]}x{blk[3]} rank {o.rank} parity {np.sqrt(nb) / np.linalg.norm(T):.2e}")
    log("C4 sampled parity", np.sqrt(pnum / den), "err", np.sqrt(num / den))
    assert np.sqrt(pnum / den) < 1e-6
    assert np.sqrt(num / den) < 10 * cfg["eps"]
    for b in rng.choice(near.shape[0], 4, replace=False):
        blk = tuple(int(v) for v in near[b])
        got = h.near_block(int(b), blk[1], blk[3])
        ref = np.transpose(op.block_tensor("slp", blk, False), (0, 2, 1))
        assert rel_fro(got, ref) < 1e-12
