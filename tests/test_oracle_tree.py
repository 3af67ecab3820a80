"""Pins for the oracle's cluster tree and block partition (invariants, brute force)."""
import numpy as np
import pytest

from inputs import cube_mesh, icosphere_mesh, lshape_mesh
from oracle import tree as T


MESHES = {
    "cube8": (cube_mesh(8), 16),
    "cube16": (cube_mesh(16), 32),
    "lshape4": (lshape_mesh(4), 16),
    "ico3": (icosphere_mesh(3), 20),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_tree_and_partition_invariants(name):
    (xyz, tri), leaf = MESHES[name]
    M = tri.shape[0]
    perm, root = T.build_tree(xyz, tri, leaf)
    assert np.array_equal(np.sort(perm), np.arange(M))
    # clusters: children split floor(n/2) / ceil(n/2), leaves <= leaf size
    stack = [root]
    while stack:
        c = stack.pop()
        ids = perm[c.start:c.start + c.size]
        vs = xyz[tri[ids].ravel()]
        assert np.array_equal(c.lo, vs.min(axis=0)) and np.array_equal(c.hi, vs.max(axis=0))
        if c.children:
            assert c.size > leaf
            a, b = c.children
            assert a.start == c.start and a.size == c.size // 2
            assert b.start == c.start + a.size and a.size + b.size == c.size
            # the split is at the median along the longest centroid axis
            cen = (xyz[tri[ids, 0]] + xyz[tri[ids, 1]] + xyz[tri[ids, 2]]) / 3.0
            ext = cen.max(axis=0) - cen.min(axis=0)
            ax = int(np.argmax(ext))
            left = cen[:a.size, ax]
            right = cen[a.size:, ax]
            assert left.max() <= right.min()
            stack += [a, b]
        else:
            assert c.size <= leaf
    far, near = T.build_partition(root, 1.0)
    cover = np.zeros((M, M), dtype=np.int32)
    for r0, m, c0, n in far + near:
        cover[r0:r0 + m, c0:c0 + n] += 1
    assert np.all(cover == 1)
    # admissibility recomputed from the vertex boxes
    def box(r0, m):
        ids = perm[r0:r0 + m]
        vs = xyz[tri[ids].ravel()]
        return vs.min(axis=0), vs.max(axis=0)
    for r0, m, c0, n in far:
        lo1, hi1 = box(r0, m)
        lo2, hi2 = box(c0, n)
        gap = np.maximum(0, np.maximum(lo1 - hi2, lo2 - hi1))
        dist = np.linalg.norm(gap)
        d1, d2 = np.linalg.norm(hi1 - lo1), np.linalg.norm(hi2 - lo2)
        assert dist > 0 and min(d1, d2) <= dist * (1 + 1e-15)
    for r0, m, c0, n in near:
        assert m <= leaf or n <= leaf


def test_diagonal_blocks_are_near():
    (xyz, tri), leaf = MESHES["cube16"]
    perm, root = T.build_tree(xyz, tri, leaf)
    far, near = T.build_partition(root, 1.0)
    for lf in T.leaves(root):
        assert (lf.start, lf.size, lf.start, lf.size) in near
