"""Oracle: cluster tree and block partition (test infrastructure only).

The paper builds its H-matrix on balanced cluster trees with a purely geometric
admissibility condition, the same partition for every frequency (Sec. 4, first
remark under "Remarks for the implementation").  It does not spell out the rules, so
this file fixes them:

* split a cluster along the longest axis of the bounding box of its element
  centroids (ties: lowest axis), at the median of a sort by (coordinate, element id);
  the left child takes the first floor(n/2) elements; a cluster of at most
  ``leaf_size`` elements is a leaf;
* a pair (sigma, tau) is admissible iff min(diam B_sigma, diam B_tau) <= eta *
  dist(B_sigma, B_tau) and the distance is positive, with B the axis-aligned box
  of the cluster's triangle vertices, diam its diagonal, dist the box-to-box distance;
* admissible -> far block; otherwise if either cluster is a leaf -> near block;
  otherwise recurse into the four child pairs (s1,t1), (s1,t2), (s2,t1), (s2,t2).

Elements are renumbered so that every cluster is a contiguous range [start, start+size).
"""
from __future__ import annotations

import numpy as np


class Cluster:
    __slots__ = ("start", "size", "lo", "hi", "children", "level")

    def __init__(self, start, size, lo, hi, level):
        self.start = start
        self.size = size
        self.lo = lo
        self.hi = hi
        self.children = []
        self.level = level

    @property
    def diam(self):
        d = self.hi - self.lo
        return float(np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]))


def centroids(xyz, tri):
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    return (a + b + c) / 3.0


def build_tree(xyz, tri, leaf_size):
    """Returns (perm, root): perm[p] = original element id at tree position p."""
    cen = centroids(xyz, tri)
    vmin = np.minimum(np.minimum(xyz[tri[:, 0]], xyz[tri[:, 1]]), xyz[tri[:, 2]])
    vmax = np.maximum(np.maximum(xyz[tri[:, 0]], xyz[tri[:, 1]]), xyz[tri[:, 2]])
    return build_tree_points(cen, vmin, vmax, leaf_size)


def build_tree_p1(xyz, tri, leaf_size):
    """Tree over the vertices (the degrees of freedom of the P1 double layer): split by
    vertex position, boxes of the supports (the triangles around each vertex), so that an
    admissible pair has well separated supports."""
    nv = xyz.shape[0]
    vmin = np.full((nv, 3), np.inf)
    vmax = np.full((nv, 3), -np.inf)
    tmin = np.minimum(np.minimum(xyz[tri[:, 0]], xyz[tri[:, 1]]), xyz[tri[:, 2]])
    tmax = np.maximum(np.maximum(xyz[tri[:, 0]], xyz[tri[:, 1]]), xyz[tri[:, 2]])
    for c in range(3):
        np.minimum.at(vmin, tri[:, c], tmin)
        np.maximum.at(vmax, tri[:, c], tmax)
    return build_tree_points(np.asarray(xyz, dtype=np.float64), vmin, vmax, leaf_size)


def build_tree_points(cen, vmin, vmax, leaf_size):
    """Tree over points cen (split coordinates) with boxes [vmin, vmax] per point."""
    perm = np.arange(cen.shape[0], dtype=np.int64)

    def make(start, size, level):
        ids = perm[start:start + size]
        lo = vmin[ids].min(axis=0)
        hi = vmax[ids].max(axis=0)
        node = Cluster(start, size, lo, hi, level)
        if size > leaf_size:
            c = cen[ids]
            ext = c.max(axis=0) - c.min(axis=0)
            axis = 0
            for k in (1, 2):
                if ext[k] > ext[axis]:
                    axis = k
            order = np.lexsort((ids, c[:, axis]))
            perm[start:start + size] = ids[order]
            half = size // 2
            node.children = [make(start, half, level + 1),
                             make(start + half, size - half, level + 1)]
        return node

    root = make(0, cen.shape[0], 0)
    return perm, root


def box_distance(s, t):
    gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
    return float(np.sqrt(gap[0] * gap[0] + gap[1] * gap[1] + gap[2] * gap[2]))


def admissible(s, t, eta):
    dist = box_distance(s, t)
    return dist > 0.0 and min(s.diam, t.diam) <= eta * dist


def build_partition(root, eta):
    """Returns (far, near): lists of (row_start, row_size, col_start, col_size)."""
    far, near = [], []

    def rec(s, t):
        if admissible(s, t, eta):
            far.append((s.start, s.size, t.start, t.size))
        elif not s.children or not t.children:
            near.append((s.start, s.size, t.start, t.size))
        else:
            for sc in s.children:
                for tc in t.children:
                    rec(sc, tc)

    rec(root, root)
    return far, near


def leaves(root):
    out = []

    def rec(c):
        if not c.children:
            out.append(c)
        for ch in c.children:
            rec(ch)

    rec(root)
    return out
