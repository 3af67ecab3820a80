"""Oracle: generalised convolution quadrature (gCQ) with Runge-Kutta time stepping, the
part that uses the compressed operators (test infrastructure only).

Paper: Sec. 3 (temporal discretisation: the ODE eq. (dgl), its Runge-Kutta solution, the
contour-integral form eq. (conv_discrete) and the algorithm with eq. (gCQ_xn) and
eq. (gcq_formula)) and App. A (integration points and weights).

* contour(dt_min, dt_max, A, n_q): App. A.  q = dt_max max|lambda(A)| / (dt_min min|lambda(A)|),
  times 5 for methods with more than one stage; k = (q - sqrt(2q - 1)) / (q + sqrt(2q - 1));
  K = K(k^2), K' = K(1 - k^2) (complete elliptic integrals in the parameter convention);
  sigma_l = -K + (l - 1/2) 4K / n_q + i K'/2, l = 1..n_q;
  s_l = gamma(sigma_l) = (sqrt(2q - 1) (1/k + sn) / (1/k - sn) - 1) / (h (q - 1));
  gamma'(sigma) = sqrt(2q - 1) / (h (q - 1)) * 2 cn dn / (k (1/k - sn)^2);
  omega_l = 4K / (2 pi i n_q) * gamma'(sigma_l),  h = dt_min min|lambda(A)|.
  Readings of the garbled passage: the weight is the trapezoidal rule of period 4K for
  (1 / 2 pi i) int_C ... ds, so it carries 1 / (2 pi i n_q) (the printed "1 pi i" has lost
  the 2 and the 1 / n_q); K' is the integral of the complementary parameter 1 - k^2; the
  printed 1 / dt_min becomes 1 / (dt_min min|lambda(A)|), so that the real segment inside the
  contour, [1 / (q h), 1 / h], holds the moduli of every pole 1 / (dt lambda_i) of
  (I - dt s A)^{-1} for dt_min <= dt <= dt_max (the two readings agree for implicit Euler,
  lambda = 1).  The points run so that sum_l omega_l F(s_l) approximates the Bromwich
  integral (1 / 2 pi i) int_{a - i inf}^{a + i inf} of eq. (conv_discrete), i.e. the
  contour closed to the right, clockwise around the poles.  The
  Jacobi functions at the complex argument come from the real ones by the addition formulas
  for an imaginary part (Abramowitz-Stegun 16.21); scipy's ellipk / ellipj are the library
  primitives for the real ones.
* history_update: eq. (gCQ_xn),
  x_{n-1}(s) = (I - dt_{n-1} s A)^{-1} ((b^T A^{-1} x_{n-2}(s)) 1 + dt_{n-1} A theta_{n-1}),
  per frequency and spatial unknown (m-vectors over the stages).
* history_weights: the vector of eq. (gcq_formula) per frequency,
  W_l = omega_l (b^T A^{-1} x_{n-1}(s_l)) (I - dt_n s_l A)^{-1} 1,
  so that the history term is sum_l V(s_l) W_l (the reordered product of Sec. 4 with the
  stages as right-hand sides).
* scalar_gcq: the whole gCQ of one scalar kernel Vhat(s) (local term by diagonalising A,
  history term by the quadrature), for the convergence pins.

Parity pins (tests/test_oracle_gcq.py): the residue theorem
sum_l omega_l F(s_l) (I - dt s_l A)^{-1} = (dt A)^{-1} F((dt A)^{-1}) for F analytic inside
the contour (exponential convergence in n_q); the real and complex Jacobi functions against
their defining identities; the scalar gCQ of a delayed pulse (the single layer kernel of one
pair of points) converges to the exact convolution as the steps shrink.
"""
from __future__ import annotations

import numpy as np
from scipy import special

# Butcher tableaux (A, b, c)
IMPLICIT_EULER = (np.array([[1.0]]), np.array([1.0]), np.array([1.0]))
RADAU_IIA_2 = (np.array([[5.0 / 12.0, -1.0 / 12.0], [3.0 / 4.0, 1.0 / 4.0]]),
               np.array([3.0 / 4.0, 1.0 / 4.0]), np.array([1.0 / 3.0, 1.0]))


def jacobi_complex(u, m):
    """sn, cn, dn of the complex argument u = x + i y for the parameter m (A-S 16.21)."""
    x, y = np.real(u), np.imag(u)
    s, c, d, _ = special.ellipj(x, m)
    s1, c1, d1, _ = special.ellipj(y, 1.0 - m)
    den = c1 ** 2 + m * s ** 2 * s1 ** 2
    sn = (s * d1 + 1j * c * d * s1 * c1) / den
    cn = (c * c1 - 1j * s * d * s1 * d1) / den
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / den
    return sn, cn, dn


def contour(dt_min: float, dt_max: float, A: np.ndarray, n_q: int):
    """Integration points s_l and weights omega_l of App. A."""
    lam = np.abs(np.linalg.eigvals(A))
    q = dt_max * lam.max() / (dt_min * lam.min())
    if A.shape[0] > 1:
        q *= 5.0
    r = np.sqrt(2.0 * q - 1.0)
    k = (q - r) / (q + r)
    m = k * k
    K, Kp = special.ellipk(m), special.ellipk(1.0 - m)
    ell = np.arange(1, n_q + 1)
    sigma = -K + (ell - 0.5) * 4.0 * K / n_q + 0.5j * Kp
    sn, cn, dn = jacobi_complex(sigma, m)
    scale = 1.0 / (dt_min * lam.min() * (q - 1.0))
    s = scale * (r * (1.0 / k + sn) / (1.0 / k - sn) - 1.0)
    gp = scale * r * 2.0 * cn * dn / (k * (1.0 / k - sn) ** 2)
    w = 4.0 * K / (2j * np.pi * n_q) * gp
    return s, w


def history_update(x2, theta1, dt1, s, A, b):
    """eq. (gCQ_xn): x_{n-1} from x_{n-2} (L x M x m), theta_{n-1} (M x m), dt_{n-1}."""
    m = A.shape[0]
    g = b @ np.linalg.inv(A)                       # b^T A^{-1}
    out = np.empty_like(x2)
    for l, sl in enumerate(s):
        Minv = np.linalg.inv(np.eye(m) - dt1 * sl * A)
        rhs = (x2[l] @ g)[:, None] * np.ones(m)[None, :] + dt1 * theta1 @ A.T
        out[l] = rhs @ Minv.T
    return out


def history_weights(x1, dt, s, w, A, b):
    """The stage vectors W_l of eq. (gcq_formula) (L x M x m) for the current step dt."""
    m = A.shape[0]
    g = b @ np.linalg.inv(A)
    out = np.empty_like(x1)
    for l, sl in enumerate(s):
        v = np.linalg.solve(np.eye(m) - dt * sl * A, np.ones(m))
        out[l] = w[l] * (x1[l] @ g)[:, None] * v[None, :]
    return out


def scalar_gcq(vhat, theta, dts, A, b, n_q):
    """gCQ of one scalar convolution (v * theta)(t) with Laplace transform vhat: returns the
    stage values (N x m) of v * theta at t_{n-1} + c dt_n.  theta(t) is a callable; the
    local term vhat((dt_n A)^{-1}) uses the eigen-decomposition of A."""
    m = A.shape[0]
    s, w = contour(min(dts), max(dts), A, n_q)
    lam, P = np.linalg.eig(A)
    Pi = np.linalg.inv(P)
    t = np.concatenate([[0.0], np.cumsum(dts)])
    cvec = A @ np.ones(m)                                  # c = A 1
    x = np.zeros((len(s), 1, m), dtype=complex)
    out = []
    th_prev = None
    for n, dt in enumerate(dts):
        th = np.array([theta(t[n] + ci * dt) for ci in cvec], dtype=complex)
        if n > 0:
            x = history_update(x, th_prev[None, :], dts[n - 1], s, A, b)
        local = P @ np.diag(vhat(1.0 / (dt * lam))) @ Pi @ th
        if n > 0:
            W = history_weights(x, dt, s, w, A, b)
            hist = np.einsum("l,lk->k", vhat(s), W[:, 0, :])
        else:
            hist = 0.0
        out.append(local + hist)
        th_prev = th
    return np.array(out)
