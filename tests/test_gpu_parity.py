"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars (FP64 path): kernel entries <= 1e-12 relative per (block, frequency) Frobenius norm;
compressed blocks ||C_gpu - C_oracle||_F / ||C||_F <= 1e-6 (expected ~1e-12 where the
pivot sequences agree), and each error against the dense tensor <= 10 eps; apply
<= 1e-12 against the dense product of the exported factors.
"""
import numpy as np
import pytest

from gpu_common import gpu_problem, log, reconstruct, rel_fro, workload

pytestmark = pytest.mark.gpu


def _oracle_problem(name):
    from oracle.hmatrix import Problem
    cfg, xyz, tri, s = workload(name)
    return cfg, Problem(xyz, tri, s, cfg["leaf"], cfg["eta"])


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_eval_entries_all_tiers(kernel):
    from oracle.entries import Geometry, collocation_entries
    log("eval entries", kernel)
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
    rng = np.random.default_rng(3)
    M, L = tri.shape[0], s.shape[0]
    n = 6000
    i = rng.integers(0, M, n)
    j = rng.integers(0, M, n)
    j[:200] = i[:200]
    # neighbours of i for the near tiers
    cen = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3
    for t in range(200, 1200):
        d = np.linalg.norm(cen - cen[i[t]], axis=1)
        j[t] = int(np.argsort(d)[1 + t % 12])
    k = rng.integers(0, L, n)
    far = (rng.random(n) < 0.3).astype(np.int32)
    far[:200] = 0
    got = prob.eval_entries(kernel, i, j, k, far)
    ref_all = collocation_entries(Geometry(xyz, tri), kernel, s, i, j, far)
    ref = ref_all[np.arange(n), k]
    scale = np.abs(ref_all).max(axis=1)
    err = np.abs(got - ref) / np.maximum(scale, 1e-300)
    err[scale == 0] = np.abs(got[scale == 0])
    log("max rel entry err", err.max())
    assert err.max() < 1e-12


def test_near_field_c1_all_entries():
    """C1 (192 triangles, leaf 16): every block is near, so the build stores the whole
    192 x 192 x 16 tensor; compare all of it with the oracle."""
    log("near C1")
    cfg, prob, _ = gpu_problem("C1")
    ocfg, op = _oracle_problem("C1")
    h = prob.build("slp")
    far, near = prob.blocks()
    assert far.shape[0] == 0 and near.shape[0] == len(op.near)
    worst = 0.0
    for b, blk in enumerate(near):
        got = h.near_block(b, int(blk[1]), int(blk[3]))          # [m][L][n]
        ref = op.block_tensor("slp", tuple(int(v) for v in blk), False)   # [m][n][L]
        ref = np.transpose(ref, (0, 2, 1))
        for l in range(ref.shape[1]):
            worst = max(worst, rel_fro(got[:, l, :], ref[:, l, :]))
    log("C1 near worst rel", worst)
    assert worst < 1e-12
    st = h.stats()
    # the 16 frequencies are 8 conjugate pairs: 8 evaluated, 8 written as conjugates
    assert st["n_far"] == 0 and st["entries_near"] == 192 * 192 * 8
    assert st["entries_near_mirrored"] == 192 * 192 * 8


def _compare_far(name, kernel, pick=None, eps_mult=10.0, **opts):
    cfg, prob, _ = gpu_problem(name, **opts)
    ocfg, op = _oracle_problem(name)
    from oracle.aca3d import aca3d
    h = prob.build(kernel)
    far, near = prob.blocks()
    idx = range(far.shape[0]) if pick is None else pick
    n_same = 0
    tot_num = tot_den = par_num = 0.0
    for b in idx:
        blk = tuple(int(v) for v in far[b])
        Tb = op.block_tensor(kernel, blk, True)
        ores = aca3d(Tb, cfg["eps"], cfg["eps_aca"])
        gb = h.export_block(b)
        C_g = reconstruct(h, b)
        C_o = ores.reconstruct(blk[1], blk[3], op.L)
        same = (gb["rank"] == ores.rank and
                all(c["k"] == oc.k and c["i"] == oc.i and c["j"] == oc.j and c["rho"] == oc.U.shape[1]
                    for c, oc in zip(gb["crosses"], ores.crosses)))
        n_same += same
        nt = np.linalg.norm(Tb)
        par_num += np.linalg.norm(C_g - C_o) ** 2
        tot_num += np.linalg.norm(C_g - Tb) ** 2
        tot_den += nt ** 2
        if nt > 0:
            assert np.linalg.norm(C_g - Tb) <= eps_mult * cfg["eps"] * nt, (b, blk)
        else:
            assert gb["rank"] == 0
    n = len(list(idx))
    par = np.sqrt(par_num / tot_den) if tot_den > 0 else np.sqrt(par_num)
    err = np.sqrt(tot_num / tot_den) if tot_den > 0 else 0.0
    log(f"{name} {kernel}: blocks {n} same pivots {n_same} parity {par:.3e} err {err:.3e}",
        h.stats())
    assert par <= 1e-6
    assert err <= eps_mult * cfg["eps"]
    return n_same, n


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_far_aca_small_all_blocks(kernel):
    log("far small", kernel)
    n_same, n = _compare_far("cube768", kernel)
    assert n_same >= 0.95 * n


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_far_aca_c2_sampled_blocks(kernel):
    log("far C2 sampled", kernel)
    cfg, prob, _ = gpu_problem("C2")
    far, _ = prob.blocks()
    rng = np.random.default_rng(17)
    pick = sorted(set(rng.choice(far.shape[0], 10, replace=False).tolist() +
                      [int(np.argmax(far[:, 1] * far[:, 3]))]))
    del prob
    n_same, n = _compare_far("C2", kernel, pick)
    assert n_same >= n - 2


@pytest.mark.parametrize("opts", [dict(threads_large=256), dict(threads_large=1024),
                                  dict(threads_small=64)], ids=["large256", "large1024", "small64"])
def test_workgroup_size_options(opts):
    """The other face-ACA workgroup sizes of the options (large faces on 256 or 1024 threads,
    the smallest faces on one wave) against the oracle on sampled C2 blocks, the largest
    block among them."""
    log("workgroup sizes", opts)
    cfg, prob, _ = gpu_problem("C2")
    far, _ = prob.blocks()
    rng = np.random.default_rng(23)
    pick = sorted(set(rng.choice(far.shape[0], 5, replace=False).tolist() +
                      [int(np.argmax(far[:, 1] * far[:, 3]))]))
    del prob
    n_same, n = _compare_far("C2", "slp", pick, **opts)
    assert n_same >= n - 1


@pytest.mark.parametrize("tl,m,n", [(1024, 700, 900), (256, 200, 240)])
def test_compress_tensor_one_entry_path_sizes(tl, m, n):
    """Faces on the one-entry-per-thread path at 1024 and 256 threads: exact reconstruction
    of a known-rank tensor with the oracle's pivots."""
    import torch
    import paper_2312_11219_amd as gaca
    from gpu_common import context
    from oracle.aca3d import aca3d
    rng = np.random.default_rng(m * n)
    L, R, rho = 5, 2, 30
    T = np.zeros((m, n, L), dtype=complex)
    for _ in range(R):
        H = (rng.standard_normal((m, rho)) + 1j * rng.standard_normal((m, rho))) @ \
            (rng.standard_normal((rho, n)) + 1j * rng.standard_normal((rho, n)))
        T += H[:, :, None] * (rng.standard_normal(L) + 1j * rng.standard_normal(L))[None, None, :]
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=1e-10, eps_aca=1e-12,
                             threads_large=tl)
    b = h.export_block(0)
    o = aca3d(T, 1e-10, 1e-12)
    err = rel_fro(reconstruct(h, 0), T)
    log(f"one-entry path {tl} threads, {m} x {n}: rank {b['rank']} (oracle {o.rank}), "
        f"face ranks {[c['rho'] for c in b['crosses']]}, rel err {err:.2e}")
    assert b["rank"] == R == o.rank
    assert err < 1e-11
    assert [c["k"] for c in b["crosses"]] == [c.k for c in o.crosses]
    assert [(c["i"], c["j"]) for c in b["crosses"]] == [(c.i, c.j) for c in o.crosses]


def test_c2_near_sampled():
    log("near C2 sampled")
    cfg, prob, _ = gpu_problem("C2")
    ocfg, op = _oracle_problem("C2")
    for kernel in ("slp", "dlp"):
        h = prob.build(kernel)
        far, near = prob.blocks()
        rng = np.random.default_rng(5)
        worst = 0.0
        for b in rng.choice(near.shape[0], 12, replace=False):
            blk = tuple(int(v) for v in near[b])
            got = h.near_block(int(b), blk[1], blk[3])
            ref = np.transpose(op.block_tensor(kernel, blk, False), (0, 2, 1))
            for l in range(ref.shape[1]):
                nr = np.linalg.norm(ref[:, l, :])
                if nr > 0:
                    worst = max(worst, np.linalg.norm(got[:, l, :] - ref[:, l, :]) / nr)
                else:
                    assert np.all(got[:, l, :] == 0)
        log("C2 near", kernel, worst)
        assert worst < 1e-12


def test_build_deterministic():
    cfg, prob, _ = gpu_problem("cube768")
    h1 = prob.build("slp")
    h2 = prob.build("slp")
    far, _ = prob.blocks()
    for b in range(0, far.shape[0], 7):
        e1, e2 = h1.export_block(b), h2.export_block(b)
        assert e1["rank"] == e2["rank"]
        for c1, c2 in zip(e1["crosses"], e2["crosses"]):
            assert np.array_equal(c1["U"], c2["U"]) and np.array_equal(c1["f"], c2["f"])


def test_problem_after_destroyed_problem():
    """A problem built after an earlier one was destroyed (it takes over that problem's
    far-field streams) gives bitwise the same operator as the first."""
    from inputs import random_rhs
    import torch
    ys = []
    for _ in range(2):
        cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
        h = prob.build("dlp")
        X = torch.from_numpy(random_rhs(cfg["L"], tri.shape[0], 3, seed=5)).cuda()
        ys.append(h.apply(X).cpu().numpy())
        del h
        prob.close()
    log("problem after a destroyed problem: max |diff|", float(np.abs(ys[0] - ys[1]).max()))
    assert np.array_equal(ys[0], ys[1])


@pytest.mark.parametrize("mode", ["sum", "per_freq"])
def test_apply_matches_exported_dense(mode):
    import torch
    from inputs import random_rhs
    log("apply", mode)
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
    h = prob.build("slp")
    far, near = prob.blocks()
    perm = prob.perm
    M, L = tri.shape[0], s.shape[0]
    C = np.zeros((M, M, L), dtype=complex)
    for b, blk in enumerate(far):
        rows = perm[blk[0]:blk[0] + blk[1]]
        cols = perm[blk[2]:blk[2] + blk[3]]
        C[np.ix_(rows, cols)] = reconstruct(h, b)
    for b, blk in enumerate(near):
        rows = perm[blk[0]:blk[0] + blk[1]]
        cols = perm[blk[2]:blk[2] + blk[3]]
        C[np.ix_(rows, cols)] = np.transpose(h.near_block(b, int(blk[1]), int(blk[3])), (0, 2, 1))
    X = random_rhs(L, M, 3, seed=4)
    Xd = torch.from_numpy(X).cuda()
    Y = h.apply(Xd, mode=mode)
    torch.cuda.synchronize()
    Y = Y.cpu().numpy()
    ref = np.einsum("ijl,ljb->ib", C, X) if mode == "sum" else np.einsum("ijl,ljb->lib", C, X)
    err = rel_fro(Y, ref)
    log("apply err", mode, err)
    assert err < 1e-12


@pytest.mark.parametrize("nrhs", [1, 2, 5])
def test_apply_sum_matches_per_freq(nrhs):
    """eq. (product) two ways on the 3072-triangle cube (far blocks of 3D rank up to 15, so
    several groups of crosses per block): the SUM apply against the PER_FREQ apply summed
    over the frequencies (separate kernels for the far part and the near rows), with 1, 2 and
    5 right-hand sides (the last one in two passes of the row kernel)."""
    import torch
    from inputs import random_rhs
    cfg, prob, (xyz, tri, s) = gpu_problem("C2")
    h = prob.build("slp")
    assert h.stats()["rank_max"] > 8
    M, L = tri.shape[0], s.shape[0]
    X = torch.from_numpy(random_rhs(L, M, nrhs, seed=21)).cuda()
    ys = h.apply(X, mode="sum")
    yf = h.apply(X, mode="per_freq")
    torch.cuda.synchronize()
    ref = yf.cpu().numpy().sum(axis=0)
    err = rel_fro(ys.cpu().numpy(), ref)
    log(f"sum vs per-frequency apply, {nrhs} rhs: {err:.3e}")
    assert err < 1e-12


def test_apply_vs_oracle_apply():
    import torch
    from inputs import random_rhs
    from oracle.hmatrix import apply as oapply, compress_far
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
    ocfg, op = _oracle_problem("cube768")
    h = prob.build("slp")
    fres = [compress_far(op, "slp", blk, cfg["eps"], cfg["eps_aca"])[0] for blk in op.far]
    ntens = [op.block_tensor("slp", blk, False) for blk in op.near]
    X = random_rhs(op.L, op.M, 2, seed=9)
    Yo = oapply(op, fres, ntens, X)
    Yg = h.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    err = rel_fro(Yg, Yo)
    log("apply vs oracle", err)
    assert err < 1e-6


@pytest.mark.parametrize("R,rho", [(1, 2), (3, 3), (6, 2)])
def test_compress_tensor_known_rank(R, rho):
    import torch
    import paper_2312_11219_amd as gaca
    from gpu_common import context
    from oracle.aca3d import aca3d
    rng = np.random.default_rng(R)
    m, n, L = 40, 33, 12
    T = np.zeros((m, n, L), dtype=complex)
    for _ in range(R):
        H = (rng.standard_normal((m, rho)) + 1j * rng.standard_normal((m, rho))) @ \
            (rng.standard_normal((rho, n)) + 1j * rng.standard_normal((rho, n)))
        T += H[:, :, None] * (rng.standard_normal(L) + 1j * rng.standard_normal(L))[None, None, :]
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=1e-10, eps_aca=1e-12)
    b = h.export_block(0)
    C = reconstruct(h, 0)
    o = aca3d(T, 1e-10, 1e-12)
    assert b["rank"] == R == o.rank
    assert rel_fro(C, T) < 1e-12
    assert [c["k"] for c in b["crosses"]] == [c.k for c in o.crosses]
    assert [(c["i"], c["j"]) for c in b["crosses"]] == [(c.i, c.j) for c in o.crosses]


@pytest.mark.parametrize("m,n", [(300, 900), (700, 1100), (1500, 420)])
def test_compress_tensor_large_faces(m, n):
    """Faces with a side above 512 (several row / column entries per thread, history mostly
    in HBM): exact reconstruction of a known-rank tensor and the oracle's pivots."""
    import torch
    import paper_2312_11219_amd as gaca
    from gpu_common import context
    from oracle.aca3d import aca3d
    rng = np.random.default_rng(m + n)
    L, R, rho = 6, 2, 12
    T = np.zeros((m, n, L), dtype=complex)
    for _ in range(R):
        H = (rng.standard_normal((m, rho)) + 1j * rng.standard_normal((m, rho))) @ \
            (rng.standard_normal((rho, n)) + 1j * rng.standard_normal((rho, n)))
        T += H[:, :, None] * (rng.standard_normal(L) + 1j * rng.standard_normal(L))[None, None, :]
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=1e-10, eps_aca=1e-12)
    b = h.export_block(0)
    o = aca3d(T, 1e-10, 1e-12)
    err = rel_fro(reconstruct(h, 0), T)
    log(f"large faces {m} x {n}: rank {b['rank']} (oracle {o.rank}), rel err {err:.2e}")
    assert b["rank"] == R == o.rank
    assert err < 1e-11
    assert [c["k"] for c in b["crosses"]] == [c.k for c in o.crosses]
    assert [(c["i"], c["j"]) for c in b["crosses"]] == [(c.i, c.j) for c in o.crosses]


@pytest.mark.parametrize("m,n,L", [(1, 1, 1), (1, 1, 5), (1, 37, 4), (37, 1, 4), (5, 64, 1),
                                   (64, 64, 2)])
def test_compress_tensor_degenerate_shapes(m, n, L):
    """Single rows, single columns, one frequency (Algorithm 1 then stops after its first
    face, every frequency used): a separable rank-1 tensor u v^T g is recovered exactly, with
    the oracle's pivots."""
    import torch
    import paper_2312_11219_amd as gaca
    from gpu_common import context
    from oracle.aca3d import aca3d
    rng = np.random.default_rng(m * 1000 + n * 10 + L)
    u = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    g = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    T = u[:, None, None] * v[None, :, None] * g[None, None, :]
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=1e-10, eps_aca=1e-12)
    b = h.export_block(0)
    o = aca3d(T, 1e-10, 1e-12)
    assert b["rank"] == o.rank == 1
    assert rel_fro(reconstruct(h, 0), T) < 1e-12
    assert [c["k"] for c in b["crosses"]] == [c.k for c in o.crosses]
    assert [(c["i"], c["j"]) for c in b["crosses"]] == [(c.i, c.j) for c in o.crosses]


def test_compress_tensor_zero_and_dense():
    import torch
    import paper_2312_11219_amd as gaca
    from gpu_common import context
    from oracle.aca3d import aca3d
    T = np.zeros((7, 5, 6), dtype=complex)
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=1e-6, eps_aca=1e-8)
    b = h.export_block(0)
    assert b["rank"] == 0 and b["zero_faces"] == 3
    rng = np.random.default_rng(1)
    T = rng.standard_normal((6, 5, 4)) + 1j * rng.standard_normal((6, 5, 4))
    h = gaca.compress_tensor(context(), torch.from_numpy(T).cuda(), eps3d=0.0, eps_aca=0.0)
    assert h.export_block(0)["rank"] == 4
    assert rel_fro(reconstruct(h, 0), T) < 1e-12
    o = aca3d(T, 0.0, 0.0)
    assert [c["k"] for c in h.export_block(0)["crosses"]] == [c.k for c in o.crosses]


def test_concurrent_builds_match_sequential():
    """Two problems built from two host threads at once give bitwise the same operators as
    the same builds one after the other."""
    from concurrent.futures import ThreadPoolExecutor
    _, p1, _ = gpu_problem("cube768")
    _, p2, _ = gpu_problem("cube768")
    seq = [p1.build("slp"), p2.build("dlp")]
    with ThreadPoolExecutor(2) as ex:
        par = list(ex.map(lambda a: a[0].build(a[1]), [(p1, "slp"), (p2, "dlp")]))
    far, _ = p1.blocks()
    for hs, hp in zip(seq, par):
        for b in range(0, far.shape[0], 7):
            es, ep = hs.export_block(b), hp.export_block(b)
            assert es["rank"] == ep["rank"]
            np.testing.assert_array_equal(reconstruct(hs, b), reconstruct(hp, b))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_joint_build_matches_separate(precision):
    """gaca_build_both gives bitwise the operators of two separate builds (the blocks of both
    operators share the far-field launches; every block's arithmetic is unchanged)."""
    import torch
    from inputs import random_rhs
    _, prob, (xyz, tri, s) = gpu_problem("cube768", precision=precision)
    sep = [prob.build("slp"), prob.build("dlp")]
    joint = prob.build_both()
    far, _ = prob.blocks()
    X = torch.from_numpy(random_rhs(len(s), tri.shape[0], 3, seed=7)).cuda()
    for hs, hj in zip(sep, joint):
        ss, sj = hs.stats(), hj.stats()
        assert sj["joint_build"] == 2 and ss["joint_build"] == 1
        for key in ("n_far", "rank_min", "rank_max", "face_rank_max", "entries_face",
                    "entries_fibre", "n_capped", "n_zero_blocks"):
            assert ss[key] == sj[key], key
        for b in range(0, far.shape[0], 5):
            es, ej = hs.export_block(b), hj.export_block(b)
            assert es["rank"] == ej["rank"]
            np.testing.assert_array_equal(reconstruct(hs, b), reconstruct(hj, b))
        ys, yj = hs.apply(X, mode="sum"), hj.apply(X, mode="sum")
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ys.cpu().numpy(), yj.cpu().numpy())
    log(f"joint build ({precision}) matches separate builds on {far.shape[0]} far blocks")


@pytest.mark.gpu
@pytest.mark.parametrize("precision,delta", [("mixed", None), ("fp64", 1e-7)])
def test_zero_row_batch_matches_one_row(precision, delta):
    """After a zero row the face ACA tries the unused rows in index order (partial-pivot ACA
    of the faces, Sec. 4).  The large-face kernels try several rows per pass over the history;
    the operator must be bitwise the one of the one-row-per-pass search.  20480-triangle
    sphere, L = 128: its mixed build walks millions of zero rows on faces of both large-face
    layouts; the FP64 case raises the zero threshold to 1e-7 to walk them in FP64 too."""
    import torch
    from inputs import random_rhs
    kw = dict(precision=precision)
    if delta is not None:
        kw["delta_zero"] = delta
    _, pb, (xyz, tri, s) = gpu_problem("C3", zero_rows_batch=1, **kw)
    _, p1, _ = gpu_problem("C3", zero_rows_batch=0, **kw)
    hb, h1 = pb.build("slp"), p1.build("slp")
    sb, s1 = hb.stats(), h1.stats()
    for key in ("n_far", "rank_min", "rank_max", "rank_mean", "face_rank_max", "face_rank_mean",
                "entries_face", "entries_fibre", "n_capped", "n_zero_blocks", "bytes_far"):
        assert sb[key] == s1[key], key
    far, _ = pb.blocks()
    for b in range(0, far.shape[0], max(1, far.shape[0] // 40)):
        assert hb.export_block(b)["rank"] == h1.export_block(b)["rank"]
    X = torch.from_numpy(random_rhs(len(s), tri.shape[0], 2, seed=11)).cuda()
    yb, y1 = hb.apply(X, mode="sum"), h1.apply(X, mode="sum")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(yb.cpu().numpy(), y1.cpu().numpy())
    log(f"zero-row batch ({precision}) matches the one-row search: {far.shape[0]} far blocks, "
        f"build {sb['ms_far']:.0f} ms vs {s1['ms_far']:.0f} ms")


def test_error_paths():
    """The boundary's error behaviour: invalid arguments come back as status codes (no
    device work is started): tensor sides outside [1, 8192], a block index out of range,
    the Galerkin double layer (unsupported), nrhs = 0."""
    import ctypes
    import torch
    import paper_2312_11219_amd as gaca
    from paper_2312_11219_amd._binding import GacaError, load_library
    from gpu_common import context
    T = torch.zeros((8193, 1, 2), dtype=torch.complex128, device="cuda")
    with pytest.raises(GacaError) as e:
        gaca.compress_tensor(context(), T)
    assert e.value.code == -1   # GACA_ERR_INVALID_ARG
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
    h = prob.build("slp")
    with pytest.raises(GacaError) as e:
        h.block_info(10 ** 9)
    assert e.value.code == -1
    lib = load_library()
    X = torch.zeros((len(s), tri.shape[0], 1), dtype=torch.complex128, device="cuda")
    Y = torch.zeros((tri.shape[0], 1), dtype=torch.complex128, device="cuda")
    rc = lib.gaca_apply(h.handle, 0, 0, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                        0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1
    _, pg, _ = gpu_problem("lshape768")
    with pytest.raises(GacaError) as e:
        pg.build("dlp")
    assert e.value.code == -6   # GACA_ERR_UNSUPPORTED
    log("error paths: invalid sides, block index, nrhs 0 and the Galerkin double layer rejected")
