"""Oracle: Galerkin operators of the Neumann problem with linear continuous test and trial
functions (test infrastructure only): the hypersingular operator D (in its form after
integration by parts) and the adjoint double layer K'.  Definition and quadrature reading:
``oracle/galerkin_p1.c``."""
from __future__ import annotations

import numpy as np

from .entries import N_MID, P1Geometry, _gauss_table, _load, _ptr, _rule6_table

OPS = {"hyp": 0, "adlp": 1}
N_GAL = 5     # collapsed rule of disjoint pairs with q < 2 (outer and each inner Duffy piece)
N_SS = 8      # Gauss points per variable of the regularising maps (touching pairs)


def p1_galerkin_entries(geom: P1Geometry, op: str, s, ii, jj, far=None, n_mid=N_MID,
                        n_gal=N_GAL, n_ss=N_SS):
    """op "hyp" (D) or "adlp" (K'): entries (ii[p], jj[p]) (vertex ids), every frequency:
    complex array (npair, L)."""
    lib = _load()
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    npair = ii.shape[0]
    far = np.zeros(npair, dtype=np.int32) if far is None else np.ascontiguousarray(far, dtype=np.int32)
    s = np.asarray(s, dtype=np.complex128)
    L = s.shape[0]
    s_re = np.ascontiguousarray(s.real)
    s_im = np.ascontiguousarray(s.imag)
    out = np.zeros((npair, L, 2), dtype=np.float64)
    r6 = _rule6_table()
    g4, gg, gs = _gauss_table(n_mid), _gauss_table(n_gal), _gauss_table(n_ss)
    lib.oracle_p1_galerkin_entries(OPS[op], _ptr(geom.xyz), _ptr(geom.tri), _ptr(geom.pptr),
                                   _ptr(geom.ptri), _ptr(geom.ploc), L, _ptr(s_re), _ptr(s_im),
                                   npair, _ptr(ii), _ptr(jj), _ptr(far), _ptr(r6), n_mid,
                                   _ptr(g4), n_gal, _ptr(gg), n_ss, _ptr(gs), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]


def pair_local(xyz, tri, kind, s, ti, tj, far=None, n_mid=N_MID, n_gal=N_GAL, n_ss=N_SS):
    """Local matrices int int k(x, y) lambda_a(x) lambda_b(y) of triangle pairs (ti[p], tj[p]):
    kind "g" (G_s) or "dnx" (dG/dn_x); complex array (npair, 3, 3, L)."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    ti = np.ascontiguousarray(ti, dtype=np.int64)
    tj = np.ascontiguousarray(tj, dtype=np.int64)
    npair = ti.shape[0]
    far = np.zeros(npair, dtype=np.int32) if far is None else np.ascontiguousarray(far, dtype=np.int32)
    s = np.asarray(s, dtype=np.complex128)
    L = s.shape[0]
    out = np.zeros((npair, 9, L, 2), dtype=np.float64)
    r6 = _rule6_table()
    g4, gg, gs = _gauss_table(n_mid), _gauss_table(n_gal), _gauss_table(n_ss)
    lib.oracle_p1_pair_local({"g": 0, "dnx": 1}[kind], _ptr(xyz), _ptr(tri), L,
                             _ptr(np.ascontiguousarray(s.real)), _ptr(np.ascontiguousarray(s.imag)),
                             npair, _ptr(ti), _ptr(tj), _ptr(far), _ptr(r6), n_mid, _ptr(g4),
                             n_gal, _ptr(gg), n_ss, _ptr(gs), _ptr(out))
    return (out[..., 0] + 1j * out[..., 1]).reshape(npair, 3, 3, L)


def ss_monomial(rel, a, b, c, d, n):
    """int int x1^a x2^b y1^c y2^d over the reference triangle pair through the regularising
    maps of relation rel (3 identical, 2 shared edge, 1 shared vertex), n points per variable."""
    return _load().oracle_ss_monomial(rel, a, b, c, d, n, _ptr(_gauss_table(n)))
