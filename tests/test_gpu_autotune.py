"""The face-ACA workgroup autotuner (options.autotune_cache): the first build of a workload
times each candidate (threads_large, threads_small) and records the choice; a later problem
of the same workload reads it from the file and builds bitwise the operator of an explicit
build with those sizes."""
import numpy as np
import pytest

from gpu_common import gpu_problem, log, reconstruct

pytestmark = pytest.mark.gpu


def test_autotune_records_and_reuses(tmp_path):
    cache = str(tmp_path / "gaca_autotune.txt")
    _, p1, _ = gpu_problem("cube768", autotune_cache=cache)
    h1 = p1.build("slp")
    s1 = h1.stats()
    assert s1["autotune_state"] == 1
    lines = open(cache).read().split("\n")
    key, tl, ts = lines[0].split()
    assert (int(tl), int(ts)) == (s1["threads_large_used"], s1["threads_small_used"])
    _, p2, _ = gpu_problem("cube768", autotune_cache=cache)
    h2 = p2.build("slp")
    s2 = h2.stats()
    assert s2["autotune_state"] == 2
    assert (s2["threads_large_used"], s2["threads_small_used"]) == (int(tl), int(ts))
    _, p3, _ = gpu_problem("cube768", threads_large=int(tl), threads_small=int(ts))
    h3 = p3.build("slp")
    far, _ = p3.blocks()
    for b in range(0, far.shape[0], 9):
        np.testing.assert_array_equal(reconstruct(h2, b), reconstruct(h3, b))
    log(f"autotune: chose threads_large {tl}, threads_small {ts} for {key}")
