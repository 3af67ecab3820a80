"""GPU tests of the mixed-precision path (FP32 far-field faces and factors with the
per-(block, frequency) scale, FP64 fibres / norms / pivots; near field FP64-computed,
FP32-stored) against the FP64 oracle and the FP64 GPU path.

Bars: each block's error against the FP64 oracle's dense tensor exceeds the FP64 path's
by at most 1e-5 (relative Frobenius, whole tensor); the FP32 apply of the mixed factors
agrees with the FP64 apply of the same factors within 1e-5; stored near field within
1e-6 of the FP64 near field.
"""
import numpy as np
import pytest

from gpu_common import gpu_problem, log, reconstruct, rel_fro, workload

pytestmark = pytest.mark.gpu


def _oracle_problem(name):
    from oracle.hmatrix import Problem
    cfg, xyz, tri, s = workload(name)
    return cfg, Problem(xyz, tri, s, cfg["leaf"], cfg["eta"])


def _errors(name, kernel, pick=None):
    cfg, p64, _ = gpu_problem(name)
    _, pmx, _ = gpu_problem(name, precision="mixed")
    ocfg, op = _oracle_problem(name)
    h64 = p64.build(kernel)
    hmx = pmx.build(kernel)
    far, near = p64.blocks()
    idx = range(far.shape[0]) if pick is None else pick
    n64 = nmx = den = 0.0
    worst_gap = 0.0
    for b in idx:
        blk = tuple(int(v) for v in far[b])
        T = op.block_tensor(kernel, blk, True)
        e64 = np.linalg.norm(reconstruct(h64, b) - T)
        emx = np.linalg.norm(reconstruct(hmx, b) - T)
        nt = np.linalg.norm(T)
        n64 += e64 ** 2
        nmx += emx ** 2
        den += nt ** 2
        if nt > 0:
            worst_gap = max(worst_gap, (emx - e64) / nt)
    e64g, emxg = np.sqrt(n64 / den), np.sqrt(nmx / den)
    log(f"{name} {kernel}: e_fp64 {e64g:.3e} e_mixed {emxg:.3e} worst block gap {worst_gap:.3e}",
        "mixed stats", {k: v for k, v in hmx.stats().items() if k.startswith(("rank", "face", "ms", "compression"))})
    return e64g, emxg, worst_gap, h64, hmx


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_mixed_small_all_blocks(kernel):
    e64, emx, gap, _, _ = _errors("cube768", kernel)
    assert emx - e64 <= 1e-5
    assert gap <= 1e-4


def test_mixed_c3_sampled_blocks():
    cfg, prob, _ = gpu_problem("C3", precision="mixed")
    far, _ = prob.blocks()
    rng = np.random.default_rng(23)
    sizes = far[:, 1] * far[:, 3]
    pick = sorted(set(rng.choice(far.shape[0], 10, replace=False).tolist() +
                      [int(np.argmax(sizes))] +
                      rng.choice(np.nonzero(sizes >= 160 * 160)[0], 3, replace=False).tolist()))
    del prob
    e64, emx, gap, h64, hmx = _errors("C3", "slp", pick)
    assert emx - e64 <= 1e-5
    assert emx <= 10 * cfg["eps"] + 1e-5


def test_mixed_near_field_stored_fp32():
    cfg, p64, _ = gpu_problem("cube768")
    _, pmx, _ = gpu_problem("cube768", precision="mixed")
    h64 = p64.build("slp")
    hmx = pmx.build("slp")
    far, near = p64.blocks()
    worst = 0.0
    for b in range(0, near.shape[0], 11):
        m, n = int(near[b, 1]), int(near[b, 3])
        a = hmx.near_block(b, m, n)
        r = h64.near_block(b, m, n)
        worst = max(worst, rel_fro(a, r))
    log("near fp32 storage rel err", worst)
    assert worst < 1e-6


@pytest.mark.parametrize("mode", ["sum", "per_freq"])
def test_mixed_apply_fp32_vs_fp64_same_factors(mode):
    import torch
    from inputs import random_rhs
    cfg, pmx, (xyz, tri, s) = gpu_problem("cube768", precision="mixed")
    h = pmx.build("slp")
    X = random_rhs(len(s), tri.shape[0], 3, seed=5)
    Y64 = h.apply(torch.from_numpy(X).cuda(), mode=mode).cpu().numpy()
    Y32 = h.apply(torch.from_numpy(X.astype(np.complex64)).cuda(), mode=mode).cpu().numpy()
    err = rel_fro(Y32.astype(np.complex128), Y64)
    log("apply fp32 vs fp64 on mixed factors", mode, err)
    assert err < 1e-5


def test_mixed_c5_sampled_blocks_and_apply():
    """The 81920-triangle sphere (L = 256, eps 1e-6) built in mixed precision as bench.py
    builds it: error against the FP64 oracle's dense tensor on seeded sampled far blocks with
    sides 64-256 (the oracle assembles each in under a second), and the matrix-core apply of
    16 right-hand sides against the FP64 VALU apply of the same operator on 8 of them."""
    import torch
    cfg, prob, (xyz, tri, s) = gpu_problem("C5", precision="mixed", batch_bytes=80 << 30)
    h = prob.build("slp")
    far, _ = prob.blocks()
    ocfg, op = _oracle_problem("C5")
    assert len(op.far) == far.shape[0]
    rng = np.random.default_rng(5)
    sizes = np.maximum(far[:, 1], far[:, 3])
    cand = np.nonzero((sizes >= 64) & (sizes <= 256))[0]
    pick = sorted(rng.choice(cand, 8, replace=False).tolist())
    num = den = 0.0
    for b in pick:
        blk = tuple(int(v) for v in far[b])
        assert blk == tuple(int(v) for v in op.far[b])
        T = op.block_tensor("slp", blk, True)
        num += np.linalg.norm(reconstruct(h, b) - T) ** 2
        den += np.linalg.norm(T) ** 2
    err = float(np.sqrt(num / den))
    M, L = tri.shape[0], len(s)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    X = torch.empty((L, M, 16), dtype=torch.complex64, device="cuda")
    X.real.normal_(generator=g)
    X.imag.normal_(generator=g)
    Y32 = h.apply(X, mode="sum")
    X64 = X[:, :, :8].to(torch.complex128).contiguous()
    del X
    Y64 = h.apply(X64, mode="sum")
    torch.cuda.synchronize()
    d = ((Y32[:, :8].to(torch.complex128) - Y64).norm() / Y64.norm()).item()
    log(f"C5 mixed: sampled blocks {pick} error vs oracle {err:.3e}; matrix-core apply vs FP64 "
        f"apply {d:.3e}; build {h.stats()['ms_total']:.0f} ms")
    assert err <= 10 * cfg["eps"] + 1e-5
    assert d <= 1e-5
