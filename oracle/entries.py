"""Oracle: Python side of the entry evaluation (test infrastructure only).

Builds ``oracle/entries.c`` with gcc (``-O2``, no fast-math, OpenMP across pairs) and
calls it through ctypes.  See entries.c for the definition and the quadrature reading.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import quadrature as Q

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "entries.c")
_SRCS = [_SRC, os.path.join(_HERE, "galerkin.c"), os.path.join(_HERE, "galerkin_p1.c")]
_LIB = os.path.join(_HERE, "_oracle_entries.so")
_lib = None

N_MID = 4    # collapsed 4 x 4 for 2 <= q < 4
N_NEAR = 8   # collapsed 8 x 8 for q < 2
N_DUFFY = 16  # Duffy order per sub-triangle of the self term


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_collocation_entries.argtypes = [
            ctypes.c_int, ctypes.c_int64, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, P,
            P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P, P]
        lib.oracle_collocation_entries.restype = None
        lib.oracle_collocation_entries_order.argtypes = [
            ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, ctypes.c_int, P, P]
        lib.oracle_collocation_entries_order.restype = None
        lib.oracle_galerkin_entries.argtypes = [
            P, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, P, P, ctypes.c_int, P,
            ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P, P]
        lib.oracle_galerkin_entries.restype = None
        lib.oracle_p1_dlp_entries.argtypes = [
            P, P, P, P, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, P, P, ctypes.c_int, P,
            ctypes.c_int, P, ctypes.c_int, P, P]
        lib.oracle_p1_dlp_entries.restype = None
        lib.oracle_p1_galerkin_entries.argtypes = [
            ctypes.c_int, P, P, P, P, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, P, P,
            ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P]
        lib.oracle_p1_galerkin_entries.restype = None
        lib.oracle_p1_pair_local.argtypes = [
            ctypes.c_int, P, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, P, P, ctypes.c_int, P,
            ctypes.c_int, P, ctypes.c_int, P, P]
        lib.oracle_p1_pair_local.restype = None
        lib.oracle_ss_monomial.argtypes = [ctypes.c_int] * 6 + [P]
        lib.oracle_ss_monomial.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _gauss_table(n):
    x, w = Q.gauss01(n)
    return np.ascontiguousarray(np.stack([x, w], axis=1))


def _rule6_table():
    p, w = Q.triangle6()
    return np.ascontiguousarray(np.concatenate([p, w[:, None]], axis=1))


KERNELS = {"slp": 0, "dlp": 1}


class Geometry:
    """Vertex coordinates of every triangle in original element order."""

    def __init__(self, xyz, tri):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.tri9 = np.ascontiguousarray(
            np.concatenate([self.xyz[self.tri[:, 0]], self.xyz[self.tri[:, 1]],
                            self.xyz[self.tri[:, 2]]], axis=1))
        self.M = self.tri.shape[0]


def collocation_entries(geom: Geometry, kernel: str, s: np.ndarray, ii, jj, far=None,
                        return_tier=False, n_mid=N_MID, n_near=N_NEAR, n_duffy=N_DUFFY):
    """E(ii[p], jj[p], l) for every l: complex array (npair, L)."""
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
    out = np.zeros((npair, L, 2), dtype=np.float64)
    tier = np.zeros(npair, dtype=np.int32)
    r6 = _rule6_table()
    g4, g8, gd = _gauss_table(n_mid), _gauss_table(n_near), _gauss_table(n_duffy)
    lib.oracle_collocation_entries(KERNELS[kernel], geom.M, _ptr(geom.tri9), L, _ptr(s_re),
                                   _ptr(s_im), npair, _ptr(ii), _ptr(jj), _ptr(far), _ptr(r6),
                                   n_mid, _ptr(g4), n_near, _ptr(g8), n_duffy, _ptr(gd),
                                   _ptr(out), _ptr(tier))
    vals = out[..., 0] + 1j * out[..., 1]
    return (vals, tier) if return_tier else vals


def collocation_entries_order(geom: Geometry, kernel: str, s, ii, jj, n):
    """Every pair with one collapsed n x n rule (self pairs: Duffy split with n x n)."""
    lib = _load()
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    L = s.shape[0]
    s_re = np.ascontiguousarray(s.real)
    s_im = np.ascontiguousarray(s.imag)
    out = np.zeros((ii.shape[0], L, 2), dtype=np.float64)
    g = _gauss_table(n)
    lib.oracle_collocation_entries_order(KERNELS[kernel], _ptr(geom.tri9), L, _ptr(s_re),
                                         _ptr(s_im), ii.shape[0], _ptr(ii), _ptr(jj), n,
                                         _ptr(g), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]


class P1Geometry:
    """Vertices and triangles of a mesh for the P1 (vertex-based) double layer: each vertex's
    patch (the triangles around it, CSR) and the vertex's local index in each triangle."""

    def __init__(self, xyz, tri):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        nv = self.xyz.shape[0]
        t = np.repeat(np.arange(self.tri.shape[0], dtype=np.int32), 3)
        v = self.tri.ravel()
        loc = np.tile(np.arange(3, dtype=np.int32), self.tri.shape[0])
        order = np.lexsort((t, v))
        self.ptri = np.ascontiguousarray(t[order])
        self.ploc = np.ascontiguousarray(loc[order])
        self.pptr = np.zeros(nv + 1, dtype=np.int64)
        np.add.at(self.pptr, v + 1, 1)
        self.pptr = np.cumsum(self.pptr)
        self.M = nv


def p1_dlp_entries(geom: P1Geometry, s, ii, jj, far=None, order=0, n_mid=N_MID, n_near=N_NEAR):
    """K(ii[p], jj[p], l) of the P1 double layer collocated at the vertices, every l:
    complex array (npair, L).  order > 0: every triangle with the collapsed order x order
    rule (the reference for the quadrature tiers)."""
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
    g4, g8 = _gauss_table(n_mid), _gauss_table(n_near)
    go = _gauss_table(max(order, 1))
    lib.oracle_p1_dlp_entries(_ptr(geom.xyz), _ptr(geom.tri), _ptr(geom.pptr), _ptr(geom.ptri),
                              _ptr(geom.ploc), L, _ptr(s_re), _ptr(s_im), npair, _ptr(ii),
                              _ptr(jj), _ptr(far), _ptr(r6), n_mid, _ptr(g4), n_near, _ptr(g8),
                              order, _ptr(go), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]
