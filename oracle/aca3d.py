"""Oracle: 3D-ACA of one block tensor C(i, j, k) (test infrastructure only).

Follows Algorithm 1 of Sec. 4 (3D-ACA) step by step, in the paper's order:

  residual face  H_l = ENTRY(:, :, k_l) - C^(l-1)(:, :, k_l),  approximated in low rank
                 by ACA on the residual face ("ACA in the faces", Sec. 4 remarks),
  pivot          (i_l, j_l) = position of the largest |H_l| found by expanding the
                 low-rank face to a dense matrix (Sec. 4 remarks, dense expansion),
  fibre          f_l[k] = (ENTRY(i_l, j_l, k) - C^(l-1)(i_l, j_l, k)) / H_l[i_l, j_l],
  update         C^(l) = C^(l-1) + H_l (x) f_l,
  norm           ||C^(l)||_F^2 by the recursion eq. (norm),
  stop           ||H_l||_F ||f_l||_2 <= eps ||C^(l)||_F,
  next frequency k_{l+1} = argmax_k |f_l[k]|.

Readings where the paper is silent or literal reading fails (all shared with the GPU
library, which implements them independently):
  * k_1 = 0; the loop body always runs once (the while-test of Algorithm 1 uses
    H_0, f_0 which are undefined);
  * the stopping cross is kept, so the stored rank r is the number of crosses;
  * the next frequency is the argmax over frequencies not used yet (taken literally,
    argmax |f_l| re-selects k_l, where f_l[k_l] = 1);
  * every argmax takes the lowest index among candidates whose squared modulus is at
    least (1 - tie)^2 times the maximum (tie = 1e-9), so that the exact ties created by
    conjugate-pair frequencies and symmetric meshes resolve the same way everywhere;
  * face ACA (partial pivoting, cited but not given in the paper): first row 0; row
    pivot j = argmax of the residual row; w = row / row[j]; u = residual column j;
    next row = argmax over unused rows of |u|; a row whose largest modulus is <= the
    zero threshold is marked used and the next unused row in index order is tried; stop
    when ||u|| ||w|| <= eps_aca sqrt(||C^(l-1)(:,:,k_l)||_F^2 + ||S||_F^2), when every row
    is used or at the face rank cap.  The face tolerance is measured against the whole
    face of the operator at s_{k_l} (the approximation so far plus the new part), not
    against the residual alone: the face is the BEM matrix at one frequency and
    eps = 100 eps_aca only keeps face errors below the 3-D tolerance on that scale.
    ||C^(l-1)(:,:,k)||_F^2 = sum_{p,q} f_p[k] conj(f_q[k]) <H_p, H_q>_F reuses the Gram
    values of eq. (norm);
  * zero faces: the zero threshold is delta * scale with scale = max over previous
    crosses of |H_p[i_p, j_p]| max_k |f_p[k]| (exact zero while no cross exists); a
    face with no usable row marks k used and moves to the lowest unused frequency;
    three consecutive zero faces, or all frequencies used, end the block.

Parity pins: tests/test_oracle_aca.py (known-rank tensors recovered exactly, eps = 0
reproduction, f_l[k_l] = 1 and f_l[k_p] = 0 on exact faces, recursion = direct norm,
error <= 10 eps on real blocks).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TIE = 1e-9
DELTA = 1e-13


def argmax_tie(a2: np.ndarray, mask: np.ndarray | None = None, tie: float = TIE) -> int:
    """Lowest index i (among mask) with a2[i] >= (1 - tie)^2 max(a2[mask])."""
    if mask is None:
        mask = np.ones(a2.shape[0], dtype=bool)
    vals = np.where(mask, a2, -1.0)
    mx = vals.max()
    thr = (1.0 - tie) ** 2 * mx
    cand = np.nonzero(mask & (a2 >= thr))[0]
    return int(cand[0])


def face_aca(R: np.ndarray, eps_aca: float, zero_tol: float, max_rank: int, tie: float = TIE,
             ref2: float = 0.0, return_pivots: bool = False):
    """Partial-pivot ACA of the dense residual face R (m x n): R ~ U W^T.  ``ref2`` is the
    squared norm of the part of the face already represented (added to ||S||^2 in the stop test).
    With ``return_pivots`` also the pivot rows and columns of the crosses, in order."""
    m, n = R.shape
    us, ws = [], []
    piv = []
    used = np.zeros(m, dtype=bool)
    s2 = 0.0
    i = 0
    while True:
        row = R[i, :].copy()
        for u, w in zip(us, ws):
            row -= u[i] * w
        used[i] = True
        a2 = row.real ** 2 + row.imag ** 2
        if np.sqrt(a2.max()) <= zero_tol:
            rest = np.nonzero(~used)[0]
            if rest.size == 0:
                break
            i = int(rest[0])
            continue
        j = argmax_tie(a2, tie=tie)
        w_new = row / row[j]
        u_new = R[:, j].copy()
        for u, w in zip(us, ws):
            u_new -= w[j] * u
        # ||S_q||^2 = ||S_{q-1}||^2 + 2 Re sum_{q'<q} <u_q,u_q'><w_q,w_q'> + |u_q|^2 |w_q|^2
        cross = 0.0
        for u, w in zip(us, ws):
            cross += (np.vdot(u, u_new) * np.vdot(w, w_new)).real
        nu2 = np.vdot(u_new, u_new).real
        nw2 = np.vdot(w_new, w_new).real
        s2 = s2 + 2.0 * cross + nu2 * nw2
        us.append(u_new)
        ws.append(w_new)
        piv.append((i, int(j)))
        if np.sqrt(nu2 * nw2) <= eps_aca * np.sqrt(ref2 + s2) or used.all() or len(us) >= max_rank:
            break
        au = u_new.real ** 2 + u_new.imag ** 2
        i = argmax_tie(au, ~used, tie=tie)
    if not us:
        U, W = np.zeros((m, 0), complex), np.zeros((n, 0), complex)
    else:
        U, W = np.stack(us, axis=1), np.stack(ws, axis=1)
    return (U, W, piv) if return_pivots else (U, W)


@dataclass
class Cross:
    k: int
    U: np.ndarray   # m x rho
    W: np.ndarray   # n x rho
    f: np.ndarray   # L
    i: int
    j: int
    hpiv: complex


@dataclass
class BlockResult:
    crosses: list = field(default_factory=list)
    used: np.ndarray = None
    zero_faces: int = 0
    capped: bool = False
    norm2: float = 0.0
    gram: list = field(default_factory=list)

    @property
    def rank(self):
        return len(self.crosses)

    def reconstruct(self, m, n, L):
        out = np.zeros((m, n, L), dtype=complex)
        for c in self.crosses:
            out += (c.U @ c.W.T)[:, :, None] * c.f[None, None, :]
        return out


def gram_face(Ua, Wa, Ub, Wb):
    """<H_a, H_b>_F = sum_ij H_a[i,j] conj(H_b[i,j]) for H = U W^T."""
    return np.sum((Ua.T @ Ub.conj()) * (Wa.T @ Wb.conj()))


def aca3d(T: np.ndarray, eps: float, eps_aca: float, max_rank3d: int | None = None,
          max_face_rank: int | None = None, tie: float = TIE, delta: float = DELTA) -> BlockResult:
    """3D-ACA of the dense block tensor T (m x n x L); ENTRY(i, j, k) = T[i, j, k]."""
    m, n, L = T.shape
    if max_rank3d is None:
        max_rank3d = L
    if max_face_rank is None:
        max_face_rank = min(m, n)
    res = BlockResult(used=np.zeros(L, dtype=bool))
    k = 0
    zero_run = 0
    norm2 = 0.0
    while True:
        # residual face at k: ENTRY(:,:,k) - C^(l-1)(:,:,k)
        R = T[:, :, k].copy()
        for c in res.crosses:
            R -= c.f[k] * (c.U @ c.W.T)
        scale = 0.0
        for c in res.crosses:
            scale = max(scale, abs(c.hpiv) * np.abs(c.f).max())
        # ||C^(l-1)(:,:,k)||_F^2 from the face Gram values and the fibres at k
        prev2 = 0.0
        for a, ca in enumerate(res.crosses):
            for b, cb in enumerate(res.crosses):
                prev2 += (ca.f[k] * np.conj(cb.f[k]) * res.gram[a][b]).real
        U, W = face_aca(R, eps_aca, delta * scale, max_face_rank, tie, ref2=max(prev2, 0.0))
        res.used[k] = True
        if U.shape[1] == 0:
            res.zero_faces += 1
            zero_run += 1
            if zero_run >= 3 or res.used.all():
                break
            k = int(np.nonzero(~res.used)[0][0])
            continue
        zero_run = 0
        H = U @ W.T
        a2 = (H.real ** 2 + H.imag ** 2).ravel()
        idx = argmax_tie(a2, tie=tie)
        i, j = divmod(idx, n)
        hpiv = H[i, j]
        f = T[i, j, :].copy()
        for c in res.crosses:
            f -= (c.U[i, :] @ c.W[j, :]) * c.f
        f = f / hpiv
        # eq. (norm): ||C^(l)||^2 = ||C^(l-1)||^2 + 2 Re sum_{p<l} <H_l,H_p><f_l,f_p> + |H_l|^2 |f_l|^2
        cross_terms = 0.0
        grow = []
        for c in res.crosses:
            g = gram_face(U, W, c.U, c.W)
            grow.append(g)
            cross_terms += (g * np.vdot(c.f, f)).real
        h2 = gram_face(U, W, U, W).real
        f2 = np.vdot(f, f).real
        norm2 = norm2 + 2.0 * cross_terms + h2 * f2
        res.crosses.append(Cross(k, U, W, f, int(i), int(j), complex(hpiv)))
        # Gram cache: gram[a][b] = <H_a, H_b>_F
        for a, g in enumerate(grow):
            res.gram[a].append(np.conj(g))
        grow.append(complex(h2))
        res.gram.append(grow)
        if np.sqrt(h2 * f2) <= eps * np.sqrt(max(norm2, 0.0)):
            break
        if res.used.all():
            break
        if len(res.crosses) >= max_rank3d:
            res.capped = True
            break
        af = f.real ** 2 + f.imag ** 2
        k = argmax_tie(af, ~res.used, tie=tie)
    res.norm2 = norm2
    return res
