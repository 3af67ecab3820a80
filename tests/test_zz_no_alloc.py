"""The allocation-free apply (gaca_apply_noalloc, workspace in the library's per-device
scratch array) against gaca_apply (allocated workspace) through the C ABI: two calls in a
row, the second with a smaller input, in both apply modes and both right-hand-side types,
and then on a second, smaller problem.  Same kernels on the same operator: the results
agree to the FP64 bar (1e-12 relative, maximum entry).  A workspace above the scratch
maximum is rejected with GACA_ERR_INVALID_ARG before any device work."""
import numpy as np
import pytest

from gpu_common import gpu_problem, log

pytestmark = pytest.mark.gpu


def _x(L, M, nrhs, seed, c64):
    import torch
    from inputs import random_rhs
    X = random_rhs(L, M, nrhs, seed=seed)
    return torch.from_numpy(X.astype(np.complex64) if c64 else X).cuda()


def _check(h, L, M, nrhs, mode, c64, seed):
    import torch
    X = _x(L, M, nrhs, seed, c64)
    y_ref = h.apply(X, mode=mode)
    y_new = h.apply(X, mode=mode, noalloc=True)
    torch.cuda.synchronize()
    a, b = y_new.cpu().numpy(), y_ref.cpu().numpy()
    d = np.abs(a - b).max() / np.abs(b).max()
    log(f"noalloc apply {mode} {'c64' if c64 else 'c128'} nrhs {nrhs}: max rel diff {d:.2e}")
    assert d <= 1e-12


@pytest.mark.parametrize("mode", ["sum", "per_freq"])
@pytest.mark.parametrize("c64", [False, True])
def test_noalloc_apply_matches_apply(mode, c64):
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768")
    h = prob.build("slp")
    L, M = len(s), tri.shape[0]
    # PER_FREQ keeps L z vectors per cross: its workspace at 2 rhs already exceeds the array
    big, small = (5, 2) if mode == "sum" else (1, 1)
    _check(h, L, M, big, mode, c64, seed=1)       # first call
    _check(h, L, M, small, mode, c64, seed=2)     # second call, smaller (or equal) input
    # a second, smaller problem (192-triangle cube) after the larger one
    cfg, p2, (xyz2, tri2, s2) = gpu_problem("C1")
    h2 = p2.build("slp")
    _check(h2, len(s2), tri2.shape[0], 1, mode, c64, seed=3)


def test_noalloc_apply_mixed_build():
    cfg, prob, (xyz, tri, s) = gpu_problem("cube768", precision="mixed")
    h = prob.build("dlp")
    _check(h, len(s), tri.shape[0], 4, "sum", True, seed=4)
    _check(h, len(s), tri.shape[0], 3, "sum", False, seed=5)


def test_noalloc_apply_rejects_large_workspace():
    import torch
    from paper_2312_11219_amd._binding import GacaError
    cfg, prob, (xyz, tri, s) = gpu_problem("C2")
    h = prob.build("slp")
    X = torch.zeros((len(s), tri.shape[0], 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(GacaError) as e:
        h.apply(X, noalloc=True)
    assert e.value.code == -1
    log("noalloc apply: a 64-rhs workspace on the 3072-triangle cube is rejected:", str(e.value))
