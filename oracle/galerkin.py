"""Oracle: Galerkin P0 single layer entries (test infrastructure only).

Python side of oracle/galerkin.c (see there for the definition and the quadrature
reading).  Tier codes: 0 far 6x6, 1 collapsed 4x4 x 4x4, 2 disjoint near (outer collapsed
+ inner nearest-point Duffy), 3 common edge and 4 common vertex (Sauter-Schwab regularising
maps, xi integral exact, n_S^3 Gauss points per region), 5 coincident (angular reduction).
"""
from __future__ import annotations

import numpy as np

from .entries import Geometry, _gauss_table, _load, _ptr, _rule6_table

N_G = 5          # outer / inner Duffy order per direction for disjoint pairs with q < 2
N_S = 12         # Gauss points per direction of the touching-pair maps (eta1, eta2, eta3)
N_THETA = 16     # Gauss points per angular sector of the coincident reduction
N_MID = 4


def galerkin_entries(geom: Geometry, kernel: str, s, ii, jj, far=None, return_tier=False,
                     n_g=N_G, n_theta=N_THETA, n_mid=N_MID, n_s=N_S):
    if kernel != "slp":
        raise ValueError("the Galerkin workload uses the single layer only")
    lib = _load()
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    npair = ii.shape[0]
    if far is None:
        far = np.zeros(npair, dtype=np.int32)
    far = np.ascontiguousarray(far, dtype=np.int32)
    s = np.asarray(s, dtype=np.complex128)
    L = s.shape[0]
    s_re = np.ascontiguousarray(s.real)
    s_im = np.ascontiguousarray(s.imag)
    out = np.zeros((npair, L, 2))
    tier = np.zeros(npair, dtype=np.int32)
    tri = np.ascontiguousarray(geom.tri, dtype=np.int32)
    lib.oracle_galerkin_entries(_ptr(geom.tri9), _ptr(tri), L, _ptr(s_re), _ptr(s_im), npair,
                                _ptr(ii), _ptr(jj), _ptr(far), _ptr(_rule6_table()), n_mid,
                                _ptr(_gauss_table(n_mid)), n_g, _ptr(_gauss_table(n_g)),
                                n_theta, _ptr(_gauss_table(n_theta)), n_s, _ptr(_gauss_table(n_s)),
                                _ptr(out), _ptr(tier))
    vals = out[..., 0] + 1j * out[..., 1]
    return (vals, tier) if return_tier else vals
