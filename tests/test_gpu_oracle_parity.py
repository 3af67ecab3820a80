"""GPU parity against the FP64 oracle for the parts that other tests compare only with the
library itself: the matrix-core apply, the mixed-precision raw far entries, per-block
compression parity, the FP64 build of the 20480-triangle sphere, the general large-face
path, and the library's device memory after every handle is destroyed.

Bars: matrix-core apply (FP32 products and sums) within 1e-5 of the oracle's eq. (product)
over the same exported factors and near blocks (maximum entry difference over maximum
entry, and relative Frobenius); mixed far entries within 1e-5 of the slice norm per (block,
frequency); FP64 blocks whose pivots agree with the oracle's within 1e-6 of ||T||_F each,
the others within 10 eps of T.
"""
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


def _exported_operator(h, far, near):
    """The operator's far blocks (as oracle cross lists) and near blocks ([m][n][L]) from the
    C-ABI export."""
    fres = [_Block(h.export_block(b)) for b in range(far.shape[0])]
    ntens = [np.transpose(h.near_block(b, int(near[b, 1]), int(near[b, 3])), (0, 2, 1))
             for b in range(near.shape[0])]
    return fres, ntens


def _x32(L, M, nrhs, seed):
    from inputs import random_rhs
    return random_rhs(L, M, nrhs, seed=seed).astype(np.complex64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [16, 64, 130])
def test_mfma_apply_vs_oracle(precision, nrhs):
    import torch
    from oracle.hmatrix import apply as oapply
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768", precision=precision)
    _, op = oracle_problem("cube768")
    h = prob.build("slp")
    far, near = prob.blocks()
    fres, ntens = _exported_operator(h, far, near)
    X = _x32(len(s), tri.shape[0], nrhs, seed=40 + nrhs)
    Y = h.apply(torch.from_numpy(X).cuda(), mode="sum")
    torch.cuda.synchronize()
    Y = Y.cpu().numpy().astype(np.complex128)
    Yo = oapply(op, fres, ntens, X.astype(np.complex128))
    emax = np.abs(Y - Yo).max() / np.abs(Yo).max()
    efro = rel_fro(Y, Yo)
    log(f"matrix-core apply vs oracle ({precision}, {nrhs} rhs): max {emax:.2e} fro {efro:.2e}")
    assert emax <= 1e-5 and efro <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mfma_apply_c2_leaf_rows_vs_oracle(precision):
    """3072-triangle cube, single layer: rows of four seeded leaf clusters of the matrix-core
    apply (16 right-hand sides) against eq. (product) evaluated by the oracle over the
    exported blocks that cover those rows."""
    import torch
    from oracle.hmatrix import apply_block_far
    cfg, prob, (xyz, tri, s) = gpu_problem("C2", precision=precision)
    h = prob.build("slp")
    far, near = prob.blocks()
    perm = prob.perm
    L, M, nrhs = len(s), tri.shape[0], 16
    X = _x32(L, M, nrhs, seed=3)
    Y = h.apply(torch.from_numpy(X).cuda(), mode="sum")
    torch.cuda.synchronize()
    Y = Y.cpu().numpy().astype(np.complex128)
    X64 = X.astype(np.complex128)
    leaves = np.unique(near[:, [0, 1]], axis=0)
    rng = np.random.default_rng(8)
    worst_max = worst_fro = 0.0
    for r0, m in leaves[rng.choice(leaves.shape[0], 4, replace=False)]:
        yr = np.zeros((m, nrhs), dtype=complex)
        for b, (b0, bm, c0, bn) in enumerate(far):
            if b0 <= r0 < b0 + bm:
                yb = apply_block_far(_Block(h.export_block(b)), X64[:, perm[c0:c0 + bn], :])
                if yb is not None:
                    yr += yb[r0 - b0:r0 - b0 + m]
        for b, (b0, bm, c0, bn) in enumerate(near):
            if b0 <= r0 < b0 + bm:
                Nb = h.near_block(b, int(bm), int(bn))     # [m][L][n]
                for l in range(L):
                    yr += Nb[r0 - b0:r0 - b0 + m, l, :] @ X64[l][perm[c0:c0 + bn]]
        got = Y[perm[r0:r0 + m]]
        worst_max = max(worst_max, np.abs(got - yr).max() / np.abs(yr).max())
        worst_fro = max(worst_fro, rel_fro(got, yr))
    log(f"C2 leaf rows, matrix-core apply vs oracle ({precision}): max {worst_max:.2e} fro {worst_fro:.2e}")
    assert worst_max <= 1e-5 and worst_fro <= 1e-5


def _far_entries_mixed_vs_oracle(name, kernel, blocks, ks):
    from oracle.entries import Geometry, collocation_entries
    from oracle.galerkin import galerkin_entries
    cfg, prob, (xyz, tri, s) = gpu_problem(name, precision="mixed")
    far, _ = prob.blocks()
    perm = prob.perm
    geom = Geometry(xyz, tri)
    worst = 0.0
    for b in blocks:
        r0, m, c0, n = (int(v) for v in far[b])
        il, jl = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
        il, jl = il.ravel(), jl.ravel()
        ii, jj = perm[r0 + il], perm[c0 + jl]
        if cfg.get("scheme") == "galerkin":
            ref = galerkin_entries(geom, kernel, s, ii, jj, np.ones(ii.shape[0], np.int32))
        else:
            ref = collocation_entries(geom, kernel, s, ii, jj, np.ones(ii.shape[0], np.int32))
        for k in ks:
            got = prob.eval_far_entries_mixed(kernel, int(b), il, jl, np.full(il.shape[0], k))
            r = ref[:, k]
            nr = np.linalg.norm(r)
            worst = max(worst, np.linalg.norm(got - r) / nr if nr > 0 else np.linalg.norm(got))
    log(f"mixed far entries vs oracle, {name} {kernel}: worst slice rel err {worst:.2e}")
    return worst


@pytest.mark.parametrize("name,kernel", [("cube768", "slp"), ("cube768", "dlp"), ("C2", "slp"),
                                         ("C2", "dlp"), ("lshape768", "slp")])
def test_mixed_far_entries_vs_oracle(name, kernel):
    _, prob, (_, _, s) = gpu_problem(name)
    far, _ = prob.blocks()
    rng = np.random.default_rng(12)
    sides = np.maximum(far[:, 1], far[:, 3])
    pick = sorted(set(rng.choice(far.shape[0], 5, replace=False).tolist() + [int(np.argmax(sides))]))
    L = len(s)
    worst = _far_entries_mixed_vs_oracle(name, kernel, pick, [0, L // 3, L // 2, L - 1])
    assert worst <= 1e-5


def _per_block_parity(name, kernel, pick, **opts):
    from oracle.aca3d import aca3d
    cfg, prob, _ = gpu_problem(name, **opts)
    _, op = oracle_problem(name)
    h = prob.build(kernel)
    far, _ = prob.blocks()
    n_same = 0
    worst_same = worst_err = 0.0
    for b in pick:
        blk = tuple(int(v) for v in far[b])
        T = op.block_tensor(kernel, blk, True)
        o = aca3d(T, cfg["eps"], cfg["eps_aca"])
        e = h.export_block(b)
        same = e["rank"] == o.rank and all(
            c["k"] == oc.k and c["i"] == oc.i and c["j"] == oc.j and c["rho"] == oc.U.shape[1]
            for c, oc in zip(e["crosses"], o.crosses))
        C = reconstruct(h, b)
        nt = np.linalg.norm(T)
        if nt == 0:
            assert e["rank"] == 0
            continue
        err = np.linalg.norm(C - T) / nt
        worst_err = max(worst_err, err)
        assert err <= 10 * cfg["eps"], (b, blk, err)
        if same:
            n_same += 1
            par = np.linalg.norm(C - o.reconstruct(blk[1], blk[3], op.L)) / nt
            worst_same = max(worst_same, par)
            assert par <= 1e-6, (b, blk, par)
    log(f"{name} {kernel} per block: {len(pick)} blocks, same pivots {n_same}, worst parity of "
        f"those {worst_same:.2e}, worst error vs T {worst_err:.2e}")
    return n_same


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_per_block_parity_cube768(kernel):
    _, prob, _ = gpu_problem("cube768")
    far, _ = prob.blocks()
    n_same = _per_block_parity("cube768", kernel, range(far.shape[0]))
    assert n_same >= 0.95 * far.shape[0]


def test_c3_fp64_vs_oracle_compression():
    """The FP64 build of the 20480-triangle sphere (L = 128, eps 1e-5) on seeded sampled far
    blocks, two of them with a side above 256, against the oracle's 3D-ACA."""
    _, prob, _ = gpu_problem("C3")
    far, _ = prob.blocks()
    side = np.maximum(far[:, 1], far[:, 3])
    rng = np.random.default_rng(29)
    pick = sorted(rng.choice(np.nonzero(side <= 256)[0], 8, replace=False).tolist()
                  + rng.choice(np.nonzero(side > 256)[0], 2, replace=False).tolist())
    del prob
    n_same = _per_block_parity("C3", "slp", pick)
    assert n_same >= len(pick) - 2


@pytest.mark.parametrize("tl,m,n", [(256, 600, 200), (512, 2700, 300)])
def test_compress_tensor_general_path(tl, m, n):
    """Faces with a side above the workgroup size (and above 2560 at 512 threads) take the
    general path of the large-face kernel: exact reconstruction of a known-rank tensor with
    the oracle's pivots."""
    import torch
    import paper_2312_11219_amd as gaca
    from oracle.aca3d import aca3d
    rng = np.random.default_rng(m + 7 * n)
    L, R, rho = 4, 2, 10
    T = np.zeros((m, n, L), dtype=complex)
    for _ in range(R):
        H = (rng.standard_normal((m, rho)) + 1j * rng.standard_normal((m, rho))) @ \
            (rng.standard_normal((rho, n)) + 1j * rng.standard_normal((rho, n)))
        T += H[:, :, None] * (rng.standard_normal(L) + 1j * rng.standard_normal(L))[None, None, :]
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=1e-10, eps_aca=1e-12,
                             threads_large=tl)
    st = h.stats()
    b = h.export_block(0)
    o = aca3d(T, 1e-10, 1e-12)
    err = rel_fro(reconstruct(h, 0), T)
    log(f"general path {tl} threads, {m} x {n}: rank {b['rank']} (oracle {o.rank}), rel err "
        f"{err:.2e}, path launches {st['launches_large_path']}")
    assert st["launches_large_path"][0] > 0
    assert b["rank"] == R == o.rank
    assert err < 1e-11
    assert [c["k"] for c in b["crosses"]] == [c.k for c in o.crosses]
    assert [(c["i"], c["j"]) for c in b["crosses"]] == [(c.i, c.j) for c in o.crosses]


def test_device_memory_returns_to_baseline():
    """Every problem and operator destroyed: the library's accounted device memory is back to
    its value before they were made, and so is the device's free memory (within 64 MiB)."""
    import gc
    import torch
    import paper_2312_11219_amd as gaca
    from inputs import random_rhs
    from gpu_common import workload
    torch.cuda.synchronize()
    ctx = gaca.Context(0)
    base = ctx.memory_in_use()
    free0 = torch.cuda.mem_get_info()[0]
    for name, precision in (("cube768", "fp64"), ("C2", "mixed"), ("lshape768", "fp64")):
        cfg, xyz, tri, s = workload(name)
        prob = gaca.Problem(ctx, xyz, tri, s, scheme=cfg.get("scheme", "collocation"),
                            leaf_size=cfg["leaf"], eta=cfg["eta"], eps3d=cfg["eps"],
                            eps_aca=cfg["eps_aca"], precision=precision)
        hs = [prob.build("slp"), prob.build("slp")]
        X = torch.from_numpy(random_rhs(len(s), tri.shape[0], 17, seed=1).astype(np.complex64)).cuda()
        for h in hs:
            h.apply(X)
        torch.cuda.synchronize()
        assert ctx.memory_in_use() > base
        del X
        for h in hs:
            h.close()
        prob.close()
        del hs, prob
        gc.collect()
        assert ctx.memory_in_use() == base, name
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    log(f"device memory: library {base} -> {ctx.memory_in_use()} bytes; device free "
        f"{free0 / 2**30:.2f} -> {free1 / 2**30:.2f} GiB")
    assert free1 >= free0 - (64 << 20)
    ctx.close()
