// Integration points and weights of the generalised convolution quadrature (gCQ), App. A:
// the contour around the poles 1 / (dt lambda_i(A)) of the Runge-Kutta resolvent
// (I - dt s A)^{-1}, dt_min <= dt <= dt_max, parametrised by Jacobi elliptic functions.
//
//   q = dt_max max|lambda| / (dt_min min|lambda|), times 5 for more than one stage,
//   k = (q - sqrt(2q - 1)) / (q + sqrt(2q - 1)), K = K(k^2), K' = K(1 - k^2) (parameter
//   convention), sigma_l = -K + (l - 1/2) 4K / n_q + i K' / 2,
//   s_l = (sqrt(2q - 1) (1/k + sn) / (1/k - sn) - 1) / (h (q - 1)),
//   omega_l = 4K / (2 pi i n_q) * sqrt(2q - 1) / (h (q - 1)) * 2 cn dn / (k (1/k - sn)^2),
//   h = dt_min min|lambda|.
// The weights make sum_l omega_l F(s_l) the quadrature of the Bromwich integral
// (1 / 2 pi i) int F ds of the convolution (Sec. 3, eq. (conv_discrete)), i.e. of the
// contour closed clockwise around the poles.  Points come in conjugate pairs
// s_{n_q - 1 - l} = conj(s_l): the first half is computed, the second half mirrored.
//
// Elliptic functions: K by the arithmetic-geometric mean, sn / cn / dn of a real argument
// by the descending Landen (AGM) recurrence (amplitude phi: sn = sin phi, cn = cos phi,
// dn = sqrt(1 - m + m cn^2)), and of a complex argument x + i y from those of
// x (parameter m) and of y (parameter 1 - m) by the addition formulas for an imaginary part.
// Eigenvalues of A: roots of its characteristic polynomial (Faddeev-LeVerrier
// coefficients, Durand-Kerner iteration).
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "host.h"
#include "internal.h"

namespace gaca {

namespace {

using cd = std::complex<double>;

double agm(double a, double b) {
    for (int it = 0; it < 64 && std::fabs(a - b) > 1e-16 * a; ++it) {
        const double an = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return a;
}

// complete elliptic integral of the first kind, parameter m in [0, 1)
double ellip_k(double m) { return M_PI / (2.0 * agm(1.0, std::sqrt(1.0 - m))); }

// sn, cn, dn of a real argument u, parameter m in [0, 1)
void jacobi_real(double u, double m, double &sn, double &cn, double &dn) {
    if (m < 1e-300) {
        sn = std::sin(u);
        cn = std::cos(u);
        dn = 1.0;
        return;
    }
    double a[32], c[32];
    a[0] = 1.0;
    double b = std::sqrt(1.0 - m);
    c[0] = std::sqrt(m);
    int n = 0;
    while (n < 30 && std::fabs(c[n]) > 1e-17) {
        a[n + 1] = 0.5 * (a[n] + b);
        c[n + 1] = 0.5 * (a[n] - b);
        b = std::sqrt(a[n] * b);
        ++n;
    }
    double phi = std::ldexp(a[n] * u, n);
    for (int j = n; j >= 1; --j) phi = 0.5 * (phi + std::asin(c[j] * std::sin(phi) / a[j]));
    sn = std::sin(phi);
    cn = std::cos(phi);
    // dn^2 = 1 - m sn^2 = (1 - m) + m cn^2: a sum of non-negative terms (no cancellation at
    // the quarter period, where the quotient form cn / cos(phi_1 - phi_0) is 0 / 0)
    dn = std::sqrt((1.0 - m) + m * cn * cn);
}

void jacobi_complex(cd u, double m, cd &sn, cd &cn, cd &dn) {
    double s, c, d, s1, c1, d1;
    jacobi_real(u.real(), m, s, c, d);
    jacobi_real(u.imag(), 1.0 - m, s1, c1, d1);
    const double den = c1 * c1 + m * s * s * s1 * s1;
    sn = cd(s * d1, c * d * s1 * c1) / den;
    cn = cd(c * c1, -s * d * s1 * d1) / den;
    dn = cd(d * c1 * d1, -m * s * c * s1) / den;
}

// moduli of the eigenvalues of the real n x n matrix A (row-major), n <= 8
void eig_moduli(int n, const double *A, double &lo, double &hi) {
    // characteristic polynomial p(z) = z^n + c[n-1] z^{n-1} + ... + c[0] (Faddeev-LeVerrier)
    std::vector<double> Mk(n * n, 0.0), AM(n * n), c(n + 1, 0.0);
    c[n] = 1.0;
    for (int k = 1; k <= n; ++k) {
        // M_k = A M_{k-1} + c_{n-k+1} I, with M_0 = 0
        std::vector<double> Mn(n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = 0.0;
                for (int t = 0; t < n; ++t) v += A[i * n + t] * Mk[t * n + j];
                Mn[i * n + j] = v + (i == j ? c[n - k + 1] : 0.0);
            }
        Mk = Mn;
        double tr = 0.0;
        for (int i = 0; i < n; ++i)
            for (int t = 0; t < n; ++t) tr += A[i * n + t] * Mk[t * n + i];
        c[n - k] = -tr / k;
    }
    // Durand-Kerner
    std::vector<cd> z(n);
    for (int i = 0; i < n; ++i) z[i] = std::pow(cd(0.4, 0.9), i);
    auto p = [&](cd x) {
        cd v = 1.0;
        for (int k = n - 1; k >= 0; --k) v = v * x + c[k];
        return v;
    };
    for (int it = 0; it < 500; ++it) {
        double delta = 0.0;
        for (int i = 0; i < n; ++i) {
            cd den = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) den *= z[i] - z[j];
            const cd dz = p(z[i]) / den;
            z[i] -= dz;
            delta = std::max(delta, std::abs(dz));
        }
        if (delta < 1e-15) break;
    }
    lo = 1e300;
    hi = 0.0;
    for (int i = 0; i < n; ++i) {
        lo = std::min(lo, std::abs(z[i]));
        hi = std::max(hi, std::abs(z[i]));
    }
}

}  // namespace

void gcq_contour(int stages, const double *rk_A, double dt_min, double dt_max, int n_q,
                 double *s_re, double *s_im, double *w_re, double *w_im) {
    // nonsingular A: |det A| against the scale max|a_ij|^stages (the characteristic
    // polynomial's constant term is (-1)^n det A)
    {
        double amax = 0.0;
        for (int i = 0; i < stages * stages; ++i) amax = std::max(amax, std::fabs(rk_A[i]));
        std::vector<double> T(rk_A, rk_A + stages * stages);
        double det = 1.0;
        for (int c = 0; c < stages; ++c) {
            int pv = c;
            for (int r = c + 1; r < stages; ++r)
                if (std::fabs(T[r * stages + c]) > std::fabs(T[pv * stages + c])) pv = r;
            if (pv != c) {
                for (int j = 0; j < stages; ++j) std::swap(T[c * stages + j], T[pv * stages + j]);
                det = -det;
            }
            det *= T[c * stages + c];
            if (T[c * stages + c] == 0.0) break;
            for (int r = c + 1; r < stages; ++r) {
                const double f = T[r * stages + c] / T[c * stages + c];
                for (int j = c; j < stages; ++j) T[r * stages + j] -= f * T[c * stages + j];
            }
        }
        if (!(std::fabs(det) > 1e-12 * std::pow(amax, stages)))
            throw Error{GACA_ERR_INVALID_ARG, "the Runge-Kutta matrix is singular"};
    }
    double lmin, lmax;
    eig_moduli(stages, rk_A, lmin, lmax);
    double q = dt_max * lmax / (dt_min * lmin);
    if (stages > 1) q *= 5.0;
    if (!(q > 1.0))
        throw Error{GACA_ERR_INVALID_ARG,
                    "q = 1 (equal steps and one stage): App. A needs q > 1, e.g. dt_max slightly above dt_min"};
    const double r = std::sqrt(2.0 * q - 1.0);
    const double k = (q - r) / (q + r);
    const double m = k * k;
    const double K = ellip_k(m), Kp = ellip_k(1.0 - m);
    const double h = dt_min * lmin;
    const double scale = 1.0 / (h * (q - 1.0));
    const int half = (n_q + 1) / 2;
    for (int l = 0; l < half; ++l) {
        const cd sigma(-K + (l + 0.5) * 4.0 * K / n_q, 0.5 * Kp);
        cd sn, cn, dn;
        jacobi_complex(sigma, m, sn, cn, dn);
        const cd s = scale * (r * (1.0 / k + sn) / (1.0 / k - sn) - 1.0);
        const cd gp = scale * r * 2.0 * cn * dn / (k * (1.0 / k - sn) * (1.0 / k - sn));
        const cd w = 4.0 * K / (cd(0.0, 2.0 * M_PI) * (double)n_q) * gp;
        s_re[l] = s.real();
        s_im[l] = s.imag();
        w_re[l] = w.real();
        w_im[l] = w.imag();
        s_re[n_q - 1 - l] = s.real();
        s_im[n_q - 1 - l] = -s.imag();
        w_re[n_q - 1 - l] = w.real();
        w_im[n_q - 1 - l] = -w.imag();
    }
    if (n_q % 2 == 1) {   // the middle point sits on the real axis
        s_im[n_q / 2] = 0.0;
        w_im[n_q / 2] = 0.0;
    }
}

}  // namespace gaca
