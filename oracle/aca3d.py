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

Recompression and pivot estimate (Sec. 4, remarks for the implementation), options of
``aca3d``:
  * recompress: after the face ACA, U W^T = Q_U (R_U R_W^T) Q_W^T with the QR factorisations
    U = Q_U R_U, W = Q_W R_W; the SVD R_U R_W^T = X Sigma Y^H gives the SVD-like form
    U' W'^T with U' = Q_U X Sigma (left singular vectors scaled) and W' = Q_W conj(Y); the
    trailing singular values are dropped while the dropped part stays within the face
    tolerance, sqrt(sum of dropped sigma^2) <= eps_aca sqrt(||C^(l-1)(:,:,k)||^2 + sum sigma^2)
    (the reference of the face ACA's own stop test), at least one kept.  H_l is the
    recompressed face.  Faces of rank 1 are already in that form and faces of rank above
    128 are kept as the face ACA left them (a bound on the work per face).
  * pivot = "index": eq. (index), the pivot estimate from the orthonormal factors,
    i = argmax_i sum_k |u_ik sigma_k| (same tie rule), then j = the largest entry of row i of
    H_l, formed from the factors (n r products); needs recompress.  Reading: taking j by the
    same estimate over the columns, independently of i, put the pivot on small entries of the
    face (their fibre divided by a near-zero value inflates ||C|| and stops the block early):
    on the 40 largest blocks of the 768-triangle cube 35 ended with errors near 1; with j
    from row i all were within 10 eps.  The default "dense" expands H_l (as the paper's
    reported results do).

Non-admissible blocks (``aca3d_dense``, Sec. 4 remarks and the "No Lwr" variant of Sec. 5):
the same algorithm with the residual face itself as H_l (no face ACA); the block is kept dense
when the compressed form would not be smaller.

Parity pins: tests/test_oracle_aca.py (known-rank tensors recovered exactly, eps = 0
reproduction, f_l[k_l] = 1 and f_l[k_p] = 0 on exact faces, recursion = direct norm,
error <= 10 eps on real blocks).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TIE = 1e-9
DELTA = 1e-13
RECOMPRESS_MAX_RANK = 128   # faces of higher rank are kept as the face ACA left them


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


def recompress(U: np.ndarray, W: np.ndarray, eps_aca: float, ref2: float = 0.0):
    """Recompressed factors (U', W', sigma) of the face U W^T (see the module header)."""
    if U.shape[1] == 0:
        return U, W, np.zeros(0)
    QU, RU = np.linalg.qr(U)
    QW, RW = np.linalg.qr(W)
    X, sig, YH = np.linalg.svd(RU @ RW.T)
    tail2 = np.cumsum((sig ** 2)[::-1])[::-1]          # tail2[k] = sum_{k' >= k} sigma_k'^2
    lim2 = eps_aca ** 2 * (ref2 + tail2[0])
    r = len(sig)
    while r > 1 and tail2[r - 1] <= lim2:
        r -= 1
    return QU @ (X[:, :r] * sig[:r]), QW @ YH[:r, :].T, sig[:r]


def index_pivot(U: np.ndarray, W: np.ndarray, sig: np.ndarray, tie: float = TIE):
    """eq. (index) for the row (U' = U_bar Sigma, so sum_k |u_ik sigma_k| = sum_k |U'_ik|),
    then the largest entry of that row of U' W'^T."""
    a = np.abs(U).sum(axis=1)
    i = argmax_tie(a * a, tie=tie)
    row = W @ U[i, :]
    return i, argmax_tie(row.real ** 2 + row.imag ** 2, tie=tie)


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
          max_face_rank: int | None = None, tie: float = TIE, delta: float = DELTA,
          recompress_faces: bool = False, pivot: str = "dense") -> BlockResult:
    """3D-ACA of the dense block tensor T (m x n x L); ENTRY(i, j, k) = T[i, j, k]."""
    if pivot not in ("dense", "index") or (pivot == "index" and not recompress_faces):
        raise ValueError("pivot must be 'dense', or 'index' with recompressed faces")
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
        sig = None
        if recompress_faces and 2 <= U.shape[1] <= RECOMPRESS_MAX_RANK:
            U, W, sig = recompress(U, W, eps_aca, ref2=max(prev2, 0.0))
        if pivot == "index":
            i, j = index_pivot(U, W, sig, tie)
            hpiv = U[i, :] @ W[j, :]
        else:
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


def aca3d_dense(T: np.ndarray, eps: float, max_rank3d: int | None = None, tie: float = TIE,
                delta: float = DELTA) -> BlockResult:
    """3D-ACA of a non-admissible block with dense faces (Sec. 4 remarks: the non-admissible
    blocks compare all their entries; Sec. 5 "No Lwr": approximation only with respect to the
    frequencies).  Algorithm 1 with H_l = the residual face ENTRY(:, :, k_l) - C^(l-1)(:, :, k_l)
    itself; pivot = largest |H_l| (tie rule), fibre, eq. (norm), stop test, next frequency and
    zero faces as in aca3d.  Each cross stores H_l as U = H_l, W = identity (so that
    reconstruct() applies unchanged)."""
    m, n, L = T.shape
    if max_rank3d is None:
        max_rank3d = L
    res = BlockResult(used=np.zeros(L, dtype=bool))
    eye = np.eye(n, dtype=complex)
    k = 0
    zero_run = 0
    norm2 = 0.0
    faces = []
    while True:
        H = T[:, :, k].copy()
        for c, Hp in zip(res.crosses, faces):
            H -= c.f[k] * Hp
        scale = 0.0
        for c in res.crosses:
            scale = max(scale, abs(c.hpiv) * np.abs(c.f).max())
        res.used[k] = True
        a2 = (H.real ** 2 + H.imag ** 2).ravel()
        if np.sqrt(a2.max()) <= delta * scale:
            res.zero_faces += 1
            zero_run += 1
            if zero_run >= 3 or res.used.all():
                break
            k = int(np.nonzero(~res.used)[0][0])
            continue
        zero_run = 0
        idx = argmax_tie(a2, tie=tie)
        i, j = divmod(idx, n)
        hpiv = H[i, j]
        f = T[i, j, :].copy()
        for c, Hp in zip(res.crosses, faces):
            f -= Hp[i, j] * c.f
        f = f / hpiv
        cross_terms = 0.0
        for c, Hp in zip(res.crosses, faces):
            g = np.sum(H * np.conj(Hp))
            cross_terms += (g * np.vdot(c.f, f)).real
        h2 = float(np.sum(a2))
        f2 = np.vdot(f, f).real
        norm2 = norm2 + 2.0 * cross_terms + h2 * f2
        res.crosses.append(Cross(k, H, eye, f, int(i), int(j), complex(hpiv)))
        faces.append(H)
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


def near_storage_compressed(m: int, n: int, L: int, rank: int, capped: bool) -> bool:
    """A non-admissible block is stored compressed when its 3D-ACA converged and
    rank (m n + L) < m n L (faces + fibres smaller than the dense block); else dense."""
    return (not capped) and rank * (m * n + L) < m * n * L
