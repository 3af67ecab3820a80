"""Pins for the oracle's gCQ (oracle/gcq.py): the Jacobi functions against their defining
identities, the contour quadrature against the residue theorem, and the scalar gCQ of a
delayed pulse against the exact convolution (convergence at the Runge-Kutta order)."""
import numpy as np
import pytest

from oracle.gcq import IMPLICIT_EULER, RADAU_IIA_2, contour, jacobi_complex, scalar_gcq


def test_jacobi_complex_identities():
    """sn^2 + cn^2 = 1, dn^2 + m sn^2 = 1 and d sn / du = cn dn (finite difference) at complex
    arguments; sn(K) = 1 and the real-axis values for zero imaginary part."""
    from scipy import special
    rng = np.random.default_rng(0)
    for m in (0.01, 0.3, 0.9, 0.999):
        u = rng.uniform(-3, 3, 20) + 1j * rng.uniform(0, 1.5, 20)
        sn, cn, dn = jacobi_complex(u, m)
        assert np.allclose(sn ** 2 + cn ** 2, 1.0, atol=1e-12)
        assert np.allclose(dn ** 2 + m * sn ** 2, 1.0, atol=1e-12)
        h = 1e-6
        sp_, _, _ = jacobi_complex(u + h, m)
        sm_, _, _ = jacobi_complex(u - h, m)
        assert np.allclose((sp_ - sm_) / (2 * h), cn * dn, rtol=1e-6, atol=1e-7)
        # complex differentiability: the derivative along i equals the one along 1
        spi, _, _ = jacobi_complex(u + 1j * h, m)
        smi, _, _ = jacobi_complex(u - 1j * h, m)
        assert np.allclose((spi - smi) / (2j * h), cn * dn, rtol=1e-6, atol=1e-7)
        sk, _, _ = jacobi_complex(np.array([special.ellipk(m) + 0j]), m)
        assert abs(sk[0] - 1.0) < 1e-12


@pytest.mark.parametrize("tab", [IMPLICIT_EULER, RADAU_IIA_2], ids=["euler", "radau2"])
def test_contour_residue_theorem(tab):
    """sum_l omega_l F(s_l) (I - dt s_l A)^{-1} -> (dt A)^{-1} F((dt A)^{-1}) (Bromwich
    integral of the resolvent: the contour closed clockwise around its poles) for F analytic
    inside the contour, dt in [dt_min, dt_max]; the error falls geometrically in n_q."""
    A, b, c = tab
    lam, P = np.linalg.eig(A)
    Pi = np.linalg.inv(P)
    F = lambda z: 1.0 / (z + 1.0) + np.exp(-0.05 * z)
    errs = []
    for nq in (64, 128, 256):
        s, w = contour(0.01, 0.1, A, nq)
        e = 0.0
        for dt in (0.01, 0.0237, 0.05, 0.1):
            ex = P @ np.diag(F(1.0 / (dt * lam)) / (dt * lam)) @ Pi
            got = sum(w[l] * F(s[l]) * np.linalg.inv(np.eye(A.shape[0]) - dt * s[l] * A)
                      for l in range(nq))
            e = max(e, np.abs(got - ex).max() / np.abs(ex).max())
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-7


def test_contour_conjugate_pairs():
    for A in (IMPLICIT_EULER[0], RADAU_IIA_2[0]):
        s, w = contour(0.02, 0.1, A, 40)
        assert np.allclose(s[::-1], np.conj(s), rtol=1e-13)
        assert np.allclose(w[::-1], np.conj(w), rtol=1e-12)
        assert np.all(s.real > 0)


@pytest.mark.parametrize("tab,order", [(IMPLICIT_EULER, 1), (RADAU_IIA_2, 3)], ids=["euler", "radau2"])
def test_scalar_gcq_converges_to_exact_convolution(tab, order):
    """v(t) = delta(t - r) / (4 pi r) (the Laplace-domain single layer e^{-s r} / (4 pi r) of
    one pair of points at distance r): (v * theta)(t) = theta(t - r) / (4 pi r).  Graded steps
    (dt_i proportional to 1 + i / N); the stage values converge at the method's order."""
    A, b, c = tab
    r = 0.5
    vhat = lambda s: np.exp(-s * r) / (4 * np.pi * r)
    theta = lambda t: t ** 5 * np.exp(-2 * t)
    errs = []
    for N in (20, 40, 80):
        T = 4.0
        g = 1.0 + np.arange(N) / N
        dts = T * g / g.sum()
        nq = int(N * np.log(N) ** 2) if A.shape[0] > 1 else int(N * np.log(N))
        out = scalar_gcq(vhat, theta, list(dts), A, b, nq)
        t = np.concatenate([[0.0], np.cumsum(dts)])
        cs = A @ np.ones(A.shape[0])
        exact = np.array([[theta(t[n] + ci * dts[n] - r) if t[n] + ci * dts[n] > r else 0.0
                           for ci in cs] for n in range(N)]) / (4 * np.pi * r)
        errs.append(np.abs(out - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > order - 0.25), (errs, rates)
