"""Oracle: block tensors, compressed H-matrix and the reordered product (test
infrastructure only).

* ``Problem`` holds the mesh, the frequencies and the cluster tree / partition.
* ``block_tensor`` assembles the dense tensor E(sigma, tau, :) of one block by the plain
  entry definition (entries.c), in tree order.
* ``compress_far`` runs Algorithm 1 (aca3d.py) on the dense tensor of an admissible block.
* ``apply`` evaluates sum_l C(s_l) X_l with the reordered product eq. (product): for every
  far block sum_k H_k (sum_l f_k[l] X_l[tau]); near blocks are dense over all frequencies.

Parity pins: tests/test_oracle_apply.py (apply = einsum over reconstructed dense blocks,
sum mode = sum of per-frequency mode), tests/test_oracle_tree.py.
"""
from __future__ import annotations

import numpy as np

from . import tree as T
from .aca3d import aca3d
from .entries import Geometry, collocation_entries


class Problem:
    """scheme: "collocation" (P0, centroids), "galerkin" (P0), "p1" (the P1 double layer
    collocated at the vertices: rows and columns are vertices) or "galerkin_p1" (the
    hypersingular operator and the adjoint double layer with P1 test and trial functions;
    n_touch points per variable of the regularising maps)."""

    def __init__(self, xyz, tri, s, leaf_size, eta, scheme="collocation", n_touch=None):
        self.s = np.asarray(s, dtype=np.complex128)
        self.L = self.s.shape[0]
        self.scheme = scheme
        self.n_touch = n_touch
        if scheme in ("p1", "galerkin_p1"):
            from .entries import P1Geometry
            self.geom = P1Geometry(xyz, tri)
            self.perm, self.root = T.build_tree_p1(self.geom.xyz, self.geom.tri, leaf_size)
        else:
            self.geom = Geometry(xyz, tri)
            self.perm, self.root = T.build_tree(self.geom.xyz, self.geom.tri, leaf_size)
        self.M = self.geom.M
        self.far, self.near = T.build_partition(self.root, eta)

    def block_ids(self, blk):
        r0, m, c0, n = blk
        return self.perm[r0:r0 + m], self.perm[c0:c0 + n]

    def block_tensor(self, kernel, blk, far):
        rows, cols = self.block_ids(blk)
        m, n = rows.shape[0], cols.shape[0]
        ii = np.repeat(rows, n)
        jj = np.tile(cols, m)
        flag = np.full(ii.shape[0], 1 if far else 0, dtype=np.int32)
        if self.scheme == "galerkin_p1":
            from .galerkin_p1 import N_SS, p1_galerkin_entries
            if kernel not in ("hyp", "adlp"):
                raise ValueError("the Galerkin P1 scheme has the hypersingular operator and the adjoint double layer")
            vals = p1_galerkin_entries(self.geom, kernel, self.s, ii, jj, flag,
                                       n_ss=self.n_touch or N_SS)
        elif self.scheme == "p1":
            from .entries import p1_dlp_entries
            if kernel != "dlp":
                raise ValueError("the P1 scheme has the double layer only")
            vals = p1_dlp_entries(self.geom, self.s, ii, jj, flag)
        elif self.scheme != "collocation":
            from .galerkin import galerkin_entries
            vals = galerkin_entries(self.geom, kernel, self.s, ii, jj, flag)
        else:
            vals = collocation_entries(self.geom, kernel, self.s, ii, jj, flag)
        return vals.reshape(m, n, self.L)

    def dense(self, kernel):
        """Full dense tensor in ORIGINAL element order (small problems only)."""
        out = np.zeros((self.M, self.M, self.L), dtype=complex)
        for blk in self.far:
            rows, cols = self.block_ids(blk)
            out[np.ix_(rows, cols)] = self.block_tensor(kernel, blk, True)
        for blk in self.near:
            rows, cols = self.block_ids(blk)
            out[np.ix_(rows, cols)] = self.block_tensor(kernel, blk, False)
        return out


def compress_far(problem: Problem, kernel: str, blk, eps: float, eps_aca: float, **kw):
    Tb = problem.block_tensor(kernel, blk, True)
    return aca3d(Tb, eps, eps_aca, **kw), Tb


def apply_block_far(res, X_tau):
    """sum_l C(:,:,l) X_l for one compressed block via eq. (product).
    X_tau: (L, n, nrhs) -> (m, nrhs)."""
    out = None
    for c in res.crosses:
        t = np.tensordot(c.f, X_tau, axes=(0, 0))       # sum_l f[l] X_l : (n, nrhs)
        y = c.U @ (c.W.T @ t)                            # H t
        out = y if out is None else out + y
    return out


def apply(problem: Problem, far_results, near_tensors, X, mode="sum"):
    """Y = sum_l C_l X_l (mode 'sum', X: L x M x nrhs -> M x nrhs) or per frequency
    (mode 'per_freq' -> L x M x nrhs), in original element order."""
    L, M, nrhs = X.shape
    if mode == "sum":
        Y = np.zeros((M, nrhs), dtype=complex)
    else:
        Y = np.zeros((L, M, nrhs), dtype=complex)
    for blk, res in zip(problem.far, far_results):
        rows, cols = problem.block_ids(blk)
        Xt = X[:, cols, :]
        if mode == "sum":
            y = apply_block_far(res, Xt)
            if y is not None:
                Y[rows] += y
        else:
            for c in res.crosses:
                H = c.U @ c.W.T
                for l in range(L):
                    Y[l][rows] += c.f[l] * (H @ Xt[l])
    for blk, Nb in zip(problem.near, near_tensors):
        rows, cols = problem.block_ids(blk)
        for l in range(L):
            y = Nb[:, :, l] @ X[l][cols]
            if mode == "sum":
                Y[rows] += y
            else:
                Y[l][rows] += y
    return Y
