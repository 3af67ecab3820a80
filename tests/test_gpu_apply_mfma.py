"""GPU tests of the matrix-core apply (SUM mode, complex64 right-hand sides, nrhs >= 16):
FP32 products on v_mfma_f32_16x16x4f32 with FP32 accumulation, against the FP64 VALU apply
of the same compressed operator (complex128 right-hand sides).  nrhs 1 and 3 are below the
matrix-core threshold and check the FP32 VALU apply the same way.  Bar: relative Frobenius
difference <= 1e-5 (FP32 rounding of factors, near field and right-hand sides, FP32 sums of
length up to L n)."""
import time

import numpy as np
import pytest

from gpu_common import gpu_problem, log, rel_fro

pytestmark = pytest.mark.gpu


def _apply_pair(h, s, M, nrhs, seed):
    import torch
    from inputs import random_rhs
    X = random_rhs(len(s), M, nrhs, seed=seed)
    X32 = torch.from_numpy(X.astype(np.complex64)).cuda()
    Y32 = h.apply(X32, mode="sum")
    torch.cuda.synchronize()
    # reference on the same (FP32-rounded) right-hand sides, FP64 arithmetic
    Y64 = h.apply(X32.to(torch.complex128), mode="sum")
    return Y32.cpu().numpy().astype(np.complex128), Y64.cpu().numpy()


@pytest.mark.parametrize("nrhs", [1, 3, 16, 64, 70, 130])
def test_mfma_apply_mixed_build(nrhs):
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768", precision="mixed")
    h = prob.build("slp")
    y32, y64 = _apply_pair(h, s, tri.shape[0], nrhs, seed=11 + nrhs)
    err = rel_fro(y32, y64)
    log(f"mfma apply mixed build nrhs {nrhs}: rel diff {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_mfma_apply_fp64_build(kernel):
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
    h = prob.build(kernel)
    y32, y64 = _apply_pair(h, s, tri.shape[0], 17, seed=5)
    err = rel_fro(y32, y64)
    log(f"mfma apply fp64 build {kernel}: rel diff {err:.3e}")
    assert err < 1e-5


def test_mfma_apply_galerkin():
    cfg, prob, (xyz, tri, s) = gpu_problem("lshape768", precision="mixed")
    h = prob.build("slp")
    y32, y64 = _apply_pair(h, s, tri.shape[0], 17, seed=2)
    err = rel_fro(y32, y64)
    log(f"mfma apply galerkin: rel diff {err:.3e}")
    assert err < 1e-5


def test_mfma_apply_c3_64rhs():
    import torch
    cfg, prob, (xyz, tri, s) = gpu_problem("C3", precision="mixed")
    h = prob.build("slp")
    st = h.stats()
    from inputs import random_rhs
    M, L, nrhs = tri.shape[0], len(s), 64
    X32 = torch.from_numpy(random_rhs(L, M, nrhs, seed=3).astype(np.complex64)).cuda()
    h.apply(X32, mode="sum")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Y32 = h.apply(X32, mode="sum")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    Y64 = h.apply(X32.to(torch.complex128), mode="sum")
    err = rel_fro(Y32.cpu().numpy().astype(np.complex128), Y64.cpu().numpy())
    gbytes = (st["bytes_far"] + st["bytes_near"]) / 1e9
    log(f"C3 mfma apply 64 rhs: {dt * 1e3:.1f} ms, stored operator {gbytes:.2f} GB "
        f"({gbytes / dt:.1f} GB/s of operator), rel diff vs FP64 apply {err:.3e}")
    assert err < 1e-5
