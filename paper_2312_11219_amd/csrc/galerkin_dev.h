// Device-side Galerkin P0 single layer entries V_ij(s) = int_{tau_i} int_{tau_j} G_s dS dS
// (Sec. 3, eq. bie_semi_indirect).  Quadrature per pair class:
//   far blocks, disjoint pairs with q >= 4:  6-point x 6-point rule
//   disjoint pairs with 2 <= q < 4:          collapsed 4x4 x collapsed 4x4
//   disjoint q < 2: outer collapsed n_G x n_G rule on tau_i (collapsed at vertex a), inner
//       integral split at the point of tau_j closest to the outer point into three Duffy
//       sub-triangles of n_G x n_G points
//   common edge, common vertex (Erichsen-Sauter / Sauter-Schwab regularising maps): both
//       triangles are parametrised over {0 <= t2 <= t1 <= 1} by P0 + t1 (P1 - P0) +
//       t2 (P2 - P1) with the shared vertex at P0 (shared edge P0 P1); the product of the two
//       parameter triangles is cut into 2 (vertex) or 5 (edge) pieces, each the image of
//       [0,1]^4 under a map (xi, eta) on which x - y = xi d(eta) (vertex) or
//       xi eta1 d(eta2, eta3) (edge), |d| bounded below.  The integrals over xi (vertex) and
//       over xi and eta1 (edge) are exact:
//         phi2(t) = int_0^1 xi^2 e^{-t xi} d xi = (2 - e^{-t} (t^2 + 2t + 2)) / t^3,
//         phie(t) = int_0^1 eta phi2(t eta) d eta = (t - 2 + e^{-t} (t + 2)) / t^3
//       (power series for |t| <= 1), the rest by n_S Gauss points per direction.  Vertex
//       order: P0, P1 the shared vertices in the order of tau_i's list (edge); each list
//       rotated to start at the shared vertex (vertex)
//   coincident: for a flat triangle the kernel depends on z = x - y only and the overlap
//       |T cap (T + z)| = A (1 - rho / R(theta))^2, so
//       V = A / (4 pi) int_0^{2 pi} R(theta) psi(s R(theta)) dtheta,
//       psi(t) = int_0^1 e^{-t u} (1 - u)^2 du; R(theta) is 1 / (G . e_theta) on each of the
//       six sectors between the edge directions (G: sum of the gradients of the barycentric
//       coordinates that grow along e_theta); n_theta Gauss points per sector.
// q = |x_i - x_j| / max(h_i, h_j).
#pragma once

#include "entries_dev.h"

namespace gaca {

enum GalTier : int32_t {
    GT_FAR36 = 0, GT_MID = 1, GT_NEAR = 2, GT_EDGE = 3, GT_VERTEX = 4, GT_COINC = 5
};

// 6 x 6 far rule at one frequency.
__device__ __forceinline__ void entry_gal36(const GeoDev &g, int64_t i, int64_t j, double sre,
                                            double sim, double &er, double &ei) {
    const int64_t M = g.M;
    double ar = 0.0, ai = 0.0;
    for (int p = 0; p < 6; ++p) {
        const double x = g.q6x[p * M + i], y = g.q6y[p * M + i], z = g.q6z[p * M + i];
        const double wx = g.q6w[p * M + i];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            double ir;
            const double r = dist3_inv(x, y, z, g.q6x[q * M + j], g.q6y[q * M + j], g.q6z[q * M + j], ir);
            kacc<0>(r, ir, sre, sim, wx * g.q6w[q * M + j], ar, ai);
        }
    }
    er = ar;
    ei = ai;
}

// Mixed precision: 6 x 6 rule divided by exp(-s d0), FP32 (same construction as the
// collocation version, with the row side also expanded into its six points).
__device__ __forceinline__ float2 entry_gal36_scaled(const GeoDev &g, float cix, float ciy,
                                                     float ciz, int64_t i, float Dx, float Dy,
                                                     float Dz, float d0, float kappa, int64_t j,
                                                     float cjx, float cjy, float cjz, float sre,
                                                     float sim) {
    const int64_t M = g.M;
    float ar = 0.0f, ai = 0.0f;
    for (int p = 0; p < 6; ++p) {
        const float ax = cix + g.q6dx[p * M + i], ay = ciy + g.q6dy[p * M + i],
                    az = ciz + g.q6dz[p * M + i];
        const float wx = g.q6wf[p * M + i];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float bx = cjx + g.q6dx[q * M + j], by = cjy + g.q6dy[q * M + j],
                        bz = cjz + g.q6dz[q * M + j];
            const float qx = ax - bx, qy = ay - by, qz = az - bz;
            const float vx = qx + Dx, vy = qy + Dy, vz = qz + Dz;
            const float r = sqrtf(vx * vx + vy * vy + vz * vz);
            const float dr =
                (2.0f * (qx * Dx + qy * Dy + qz * Dz) + (qx * qx + qy * qy + qz * qz) + kappa) / (r + d0);
            const float mag = expf(-sre * dr);
            float sn, cs;
            sincosf(sim * dr, &sn, &cs);
            const float c = wx * g.q6wf[q * M + j] / (12.566370614359172f * r);
            ar += c * mag * cs;
            ai -= c * mag * sn;
        }
    }
    return make_float2(ar, ai);
}

// Closest point of the triangle (a, b, c) to x: projection onto the plane if it lies
// inside, otherwise the nearest of the three clamped edge projections.
__device__ __forceinline__ void closest_on_triangle(const double *x, const double *a,
                                                    const double *b, const double *c,
                                                    double *out) {
    double e0[3], e1[3], d[3];
    for (int k = 0; k < 3; ++k) {
        e0[k] = b[k] - a[k];
        e1[k] = c[k] - a[k];
        d[k] = x[k] - a[k];
    }
    const double a00 = e0[0] * e0[0] + e0[1] * e0[1] + e0[2] * e0[2];
    const double a01 = e0[0] * e1[0] + e0[1] * e1[1] + e0[2] * e1[2];
    const double a11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const double b0 = e0[0] * d[0] + e0[1] * d[1] + e0[2] * d[2];
    const double b1 = e1[0] * d[0] + e1[1] * d[1] + e1[2] * d[2];
    const double det = a00 * a11 - a01 * a01;
    const double u = (a11 * b0 - a01 * b1) / det, v = (a00 * b1 - a01 * b0) / det;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
        for (int k = 0; k < 3; ++k) out[k] = a[k] + u * e0[k] + v * e1[k];
        return;
    }
    const double *P[3] = {a, b, c};
    double best = 1e300;
    for (int e = 0; e < 3; ++e) {
        const double *p0 = P[e], *p1 = P[(e + 1) % 3];
        double s[3], w[3];
        for (int k = 0; k < 3; ++k) {
            s[k] = p1[k] - p0[k];
            w[k] = x[k] - p0[k];
        }
        double t = (s[0] * w[0] + s[1] * w[1] + s[2] * w[2]) / (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        t = fmin(1.0, fmax(0.0, t));
        double cpt[3], dd = 0.0;
        for (int k = 0; k < 3; ++k) {
            cpt[k] = p0[k] + t * s[k];
            dd += (x[k] - cpt[k]) * (x[k] - cpt[k]);
        }
        if (dd < best) {
            best = dd;
            out[0] = cpt[0];
            out[1] = cpt[1];
            out[2] = cpt[2];
        }
    }
}

// Inner integral over tau_j at x (split at the closest point), accumulated with weight wx.
template <int NF>
__device__ __forceinline__ void gal_inner_split(const double *x, double wx, const double *a,
                                                const double *b, const double *c, int n,
                                                const double *gt, const FreqDev &f, int l0,
                                                int nl, double *ar, double *ai) {
    double p[3];
    closest_on_triangle(x, a, b, c, p);
    const double *V[3] = {a, b, c};
    for (int s = 0; s < 3; ++s) {
        const double *p1 = V[(s + 1) % 3], *p2 = V[(s + 2) % 3];
        double e1x = p1[0] - p[0], e1y = p1[1] - p[1], e1z = p1[2] - p[2];
        double e2x = p2[0] - p1[0], e2y = p2[1] - p1[1], e2z = p2[2] - p1[2];
        double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
        const double two_area = sqrt(nx * nx + ny * ny + nz * nz);
        if (two_area == 0.0) continue;
        for (int iu = 0; iu < n; ++iu) {
            const double u = gt[2 * iu], wu = gt[2 * iu + 1];
            for (int iv = 0; iv < n; ++iv) {
                const double v = gt[2 * iv], wv = gt[2 * iv + 1];
                const double uv = u * v;
                double ir;
                const double r = dist3_inv(x[0], x[1], x[2], p[0] + u * e1x + uv * e2x,
                                           p[1] + u * e1y + uv * e2y, p[2] + u * e1z + uv * e2z, ir);
                const double w = wx * wu * wv * u * two_area;
#pragma unroll
                for (int t = 0; t < NF; ++t)
                    if (t < nl) kacc<0>(r, ir, f.re[l0 + t], f.im[l0 + t], w, ar[t], ai[t]);
            }
        }
    }
}

// psi(t) = int_0^1 e^{-t u} (1 - u)^2 du for complex t.
__device__ __forceinline__ double2 gal_psi(double tr, double ti) {
    const double at = sqrt(tr * tr + ti * ti);
    if (at < 2.0) {
        // 2 sum_k (-t)^k / (k + 3)!, Horner from k = 39 down
        double cr = 0.0, ci = 0.0;
        double fact = 1.0;
        for (int k = 1; k <= 42; ++k) fact *= k;   // 42! = (39 + 3)!
        for (int k = 39; k >= 0; --k) {
            // c = c * (-t) + 2 / (k + 3)!
            const double nr = -(cr * tr - ci * ti), ni = -(cr * ti + ci * tr);
            cr = nr + 2.0 / fact;
            ci = ni;
            fact /= (k + 3);
        }
        return make_double2(cr, ci);
    }
    // 1/t - 2/t^2 + 2/t^3 - 2 e^{-t}/t^3
    const double d = tr * tr + ti * ti;
    const double ir = tr / d, ii = -ti / d;                      // 1/t
    const double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;   // 1/t^2
    const double i3r = i2r * ir - i2i * ii, i3i = i2r * ii + i2i * ir;
    const double m = fm::exp(-tr);
    double sn, cs;
    fm::sincos(ti, &sn, &cs);
    const double er = m * cs, ei = -m * sn;                      // e^{-t}
    const double qr = er * i3r - ei * i3i, qi = er * i3i + ei * i3r;
    return make_double2(ir - 2.0 * i2r + 2.0 * i3r - 2.0 * qr, ii - 2.0 * i2i + 2.0 * i3i - 2.0 * qi);
}

// Coincident Galerkin entry by the angular reduction, NF frequencies from l0.
template <int NF>
__device__ void gal_coincident(const double *a, const double *b, const double *c, int nth,
                               const double *gt, const FreqDev &f, int l0, int nl, double *ar,
                               double *ai) {
    // orthonormal in-plane frame at a
    double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    const double lu = sqrt(ux * ux + uy * uy + uz * uz);
    ux /= lu; uy /= lu; uz /= lu;
    double wx = c[0] - a[0], wy = c[1] - a[1], wz = c[2] - a[2];
    const double wu = wx * ux + wy * uy + wz * uz;
    double vx = wx - wu * ux, vy = wy - wu * uy, vz = wz - wu * uz;
    const double lv = sqrt(vx * vx + vy * vy + vz * vz);
    vx /= lv; vy /= lv; vz /= lv;
    // 2-D vertices: (0, 0), (lu, 0), (wu, lv)
    const double P[3][2] = {{0.0, 0.0}, {lu, 0.0}, {wu, lv}};
    const double area = 0.5 * lu * lv;
    const double A2 = 2.0 * area;
    double Gx[3], Gy[3];
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        Gx[k] = (P[k1][1] - P[k2][1]) / A2;
        Gy[k] = (P[k2][0] - P[k1][0]) / A2;
    }
    // sector boundaries: the three edge directions and their opposites
    double th[6];
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3;
        double t = atan2(P[k1][1] - P[k][1], P[k1][0] - P[k][0]);
        if (t < 0.0) t += 2.0 * M_PI;
        th[2 * k] = t;
        double t2 = t + M_PI;
        if (t2 >= 2.0 * M_PI) t2 -= 2.0 * M_PI;
        th[2 * k + 1] = t2;
    }
    for (int x = 1; x < 6; ++x)
        for (int y = x; y > 0 && th[y] < th[y - 1]; --y) {
            const double tmp = th[y];
            th[y] = th[y - 1];
            th[y - 1] = tmp;
        }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] = 0.0;
        ai[t] = 0.0;
    }
    for (int sct = 0; sct < 6; ++sct) {
        const double ta = th[sct], tb = sct == 5 ? th[0] + 2.0 * M_PI : th[sct + 1];
        const double span = tb - ta;
        if (span <= 0.0) continue;
        for (int q = 0; q < nth; ++q) {
            const double theta = ta + span * gt[2 * q];
            const double wq = span * gt[2 * q + 1];
            double sn, cs;
            sincos(theta, &sn, &cs);
            double gsum = 0.0;
            for (int k = 0; k < 3; ++k) gsum += fmax(0.0, Gx[k] * cs + Gy[k] * sn);
            const double R = 1.0 / gsum;
#pragma unroll
            for (int t = 0; t < NF; ++t)
                if (t < nl) {
                    const double2 ps = gal_psi(f.re[l0 + t] * R, f.im[l0 + t] * R);
                    ar[t] += wq * R * ps.x;
                    ai[t] += wq * R * ps.y;
                }
        }
    }
    const double sc = area / kFourPi;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] *= sc;
        ai[t] *= sc;
    }
}


// Power-series coefficients of phi2 (1 / (k! (k + 3))) and phie (1 / (k! (k + 2) (k + 3))).
struct SsSeries {
    double c2[20], ce[20];
};
constexpr SsSeries make_ss_series() {
    SsSeries t{};
    double fact = 1.0;
    for (int k = 0; k < 20; ++k) {
        if (k > 0) fact *= k;
        t.c2[k] = 1.0 / (fact * (k + 3));
        t.ce[k] = 1.0 / (fact * (k + 2) * (k + 3));
    }
    return t;
}

// EDGE = false: phi2(t); true: phie(t).  t = tr + i ti.
template <bool EDGE>
__device__ __forceinline__ double2 ss_phi(double tr, double ti) {
    constexpr SsSeries S = make_ss_series();
    if (tr * tr + ti * ti <= 1.0) {
        // sum_k c_k (-t)^k by Horner from k = 19
        double cr = EDGE ? S.ce[19] : S.c2[19], ci = 0.0;
#pragma unroll
        for (int k = 18; k >= 0; --k) {
            const double nr = -(cr * tr - ci * ti), ni = -(cr * ti + ci * tr);
            cr = nr + (EDGE ? S.ce[k] : S.c2[k]);
            ci = ni;
        }
        return make_double2(cr, ci);
    }
    const double m = fm::exp(-tr);
    double sn, cs;
    fm::sincos(ti, &sn, &cs);
    const double er = m * cs, ei = -m * sn;   // e^{-t}
    double nr, ni;                            // numerator
    if (EDGE) {
        // t - 2 + e^{-t} (t + 2)
        const double ar = tr + 2.0;
        nr = tr - 2.0 + (er * ar - ei * ti);
        ni = ti + (er * ti + ei * ar);
    } else {
        // 2 - e^{-t} (t^2 + 2 t + 2)
        const double pr = tr * tr - ti * ti + 2.0 * tr + 2.0, pi = 2.0 * tr * ti + 2.0 * ti;
        nr = 2.0 - (er * pr - ei * pi);
        ni = -(er * pi + ei * pr);
    }
    // / t^3
    const double t2r = tr * tr - ti * ti, t2i = 2.0 * tr * ti;
    const double t3r = t2r * tr - t2i * ti, t3i = t2r * ti + t2i * tr;
    const double den = t3r * t3r + t3i * t3i;
    return make_double2((nr * t3r + ni * t3i) / den, (ni * t3r - nr * t3i) / den);
}

// w * phi(s_l rho) / (4 pi rho) added for the thread's frequencies
template <bool EDGE, int NF>
__device__ __forceinline__ void ss_acc(const double *d, double w, const FreqDev &f, int l0, int nl,
                                       double *ar, double *ai) {
    const double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double c = w / (kFourPi * rho);
#pragma unroll
    for (int t = 0; t < NF; ++t)
        if (t < nl) {
            const double2 ph = ss_phi<EDGE>(f.re[l0 + t] * rho, f.im[l0 + t] * rho);
            ar[t] += c * ph.x;
            ai[t] += c * ph.y;
        }
}

// Common vertex V: tau_i = (V, a1, a2), tau_j = (V, b1, b2).
template <int NF>
__device__ void gal_ss_vertex(const double *V, const double *a1, const double *a2,
                              const double *b1, const double *b2, double area_i, double area_j,
                              int n, const double *g, const FreqDev &f, int l0, int nl,
                              double *ar, double *ai) {
    double X1[3], X2[3], Y1[3], Y2[3];
    for (int k = 0; k < 3; ++k) {
        X1[k] = a1[k] - V[k];
        X2[k] = a2[k] - a1[k];
        Y1[k] = b1[k] - V[k];
        Y2[k] = b2[k] - b1[k];
    }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] = 0.0;
        ai[t] = 0.0;
    }
    for (int p1 = 0; p1 < n; ++p1) {
        const double e1 = g[2 * p1], w1 = g[2 * p1 + 1];
        for (int p2 = 0; p2 < n; ++p2) {
            const double e2 = g[2 * p2], w12 = w1 * g[2 * p2 + 1];
            for (int p3 = 0; p3 < n; ++p3) {
                const double e3 = g[2 * p3], w = w12 * g[2 * p3 + 1] * e2;
                double d[3];
                // t1 >= u1: t = xi (1, e1), u = xi e2 (1, e3)
                for (int k = 0; k < 3; ++k) d[k] = (X1[k] + e1 * X2[k]) - e2 * (Y1[k] + e3 * Y2[k]);
                ss_acc<false, NF>(d, w, f, l0, nl, ar, ai);
                // u1 > t1: u = xi (1, e1), t = xi e2 (1, e3)
                for (int k = 0; k < 3; ++k) d[k] = e2 * (X1[k] + e3 * X2[k]) - (Y1[k] + e1 * Y2[k]);
                ss_acc<false, NF>(d, w, f, l0, nl, ar, ai);
            }
        }
    }
    const double sc = 4.0 * area_i * area_j;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] *= sc;
        ai[t] *= sc;
    }
}

// Common edge (P0, P1): tau_i = (P0, P1, a), tau_j = (P0, P1, b).
template <int NF>
__device__ void gal_ss_edge(const double *P0, const double *P1, const double *a, const double *b,
                            double area_i, double area_j, int n, const double *g,
                            const FreqDev &f, int l0, int nl, double *ar, double *ai) {
    double E[3], A[3], B[3];
    for (int k = 0; k < 3; ++k) {
        E[k] = P1[k] - P0[k];
        A[k] = a[k] - P1[k];
        B[k] = b[k] - P1[k];
    }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] = 0.0;
        ai[t] = 0.0;
    }
    for (int p2 = 0; p2 < n; ++p2) {
        const double e2 = g[2 * p2], w2 = g[2 * p2 + 1];
        for (int p3 = 0; p3 < n; ++p3) {
            const double e3 = g[2 * p3], w = w2 * g[2 * p3 + 1];
            // coefficients of (E, A, B) in d for the five pieces
            const double c[5][3] = {{e2, e3, -(1.0 - e2)},
                                    {e2 * e3, 1.0, -e2 * (1.0 - e3)},
                                    {-e2, 1.0 - e2, -e2 * e3},
                                    {-e2 * e3, e2 * (1.0 - e3), -1.0},
                                    {-e2 * e3, 1.0 - e2 * e3, -e2}};
#pragma unroll
            for (int r = 0; r < 5; ++r) {
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = c[r][0] * E[k] + c[r][1] * A[k] + c[r][2] * B[k];
                ss_acc<true, NF>(d, r == 0 ? w : w * e2, f, l0, nl, ar, ai);
            }
        }
    }
    const double sc = 4.0 * area_i * area_j;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] *= sc;
        ai[t] *= sc;
    }
}

// Near-block Galerkin entry of pair (i, j) (tree positions) with the given class.
template <int NF>
__device__ void gal_near_entry(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t i,
                               int64_t j, int tier, int l0, int nl, double *ar, double *ai) {
    const double ai3[3][3] = {{g.ax[i], g.ay[i], g.az[i]}, {g.bx[i], g.by[i], g.bz[i]},
                              {g.cx[i], g.cy[i], g.cz[i]}};
    const double aj[3] = {g.ax[j], g.ay[j], g.az[j]};
    const double bj[3] = {g.bx[j], g.by[j], g.bz[j]};
    const double cj[3] = {g.cx[j], g.cy[j], g.cz[j]};
    if (tier == GT_COINC) {
        gal_coincident<NF>(aj, bj, cj, q.nth, q.gth, f, l0, nl, ar, ai);
        return;
    }
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] = 0.0;
        ai[t] = 0.0;
    }
    if (tier == GT_FAR36) {
        const int64_t M = g.M;
        for (int p = 0; p < 6; ++p) {
            const double x = g.q6x[p * M + i], y = g.q6y[p * M + i], z = g.q6z[p * M + i];
            const double wx = g.q6w[p * M + i];
            for (int qq = 0; qq < 6; ++qq) {
                double ir;
                const double r =
                    dist3_inv(x, y, z, g.q6x[qq * M + j], g.q6y[qq * M + j], g.q6z[qq * M + j], ir);
                const double w = wx * g.q6w[qq * M + j];
#pragma unroll
                for (int t = 0; t < NF; ++t)
                    if (t < nl) kacc<0>(r, ir, f.re[l0 + t], f.im[l0 + t], w, ar[t], ai[t]);
            }
        }
        return;
    }
    if (tier == GT_EDGE || tier == GT_VERTEX) {
        // shared vertices (equal coordinates): positions in tau_i (ascending) and tau_j
        const double *Vj[3] = {aj, bj, cj};
        int ns = 0, pi_[3] = {0, 0, 0}, pj_[3] = {0, 0, 0};
        for (int va = 0; va < 3; ++va)
            for (int vb = 0; vb < 3; ++vb)
                if (ai3[va][0] == Vj[vb][0] && ai3[va][1] == Vj[vb][1] && ai3[va][2] == Vj[vb][2]) {
                    pi_[ns] = va;
                    pj_[ns] = vb;
                    ++ns;
                }
        if (tier == GT_EDGE) {
            gal_ss_edge<NF>(ai3[pi_[0]], ai3[pi_[1]], ai3[3 - pi_[0] - pi_[1]],
                            Vj[3 - pj_[0] - pj_[1]], g.area[i], g.area[j], q.ns, q.gs, f, l0, nl,
                            ar, ai);
        } else {
            const int a = pi_[0], b = pj_[0];
            gal_ss_vertex<NF>(ai3[a], ai3[(a + 1) % 3], ai3[(a + 2) % 3], Vj[(b + 1) % 3],
                              Vj[(b + 2) % 3], g.area[i], g.area[j], q.ns, q.gs, f, l0, nl, ar, ai);
        }
        return;
    }
    const int c0 = 0;
    const double *A0 = ai3[c0], *A1 = ai3[(c0 + 1) % 3], *A2 = ai3[(c0 + 2) % 3];
    const int no = tier == GT_MID ? q.n4 : q.ng;
    const double *go = tier == GT_MID ? q.g4 : q.gg;
    double e1x = A1[0] - A0[0], e1y = A1[1] - A0[1], e1z = A1[2] - A0[2];
    double e2x = A2[0] - A1[0], e2y = A2[1] - A1[1], e2z = A2[2] - A1[2];
    double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const double two_area = sqrt(nx * nx + ny * ny + nz * nz);
    for (int iu = 0; iu < no; ++iu) {
        const double u = go[2 * iu], wu = go[2 * iu + 1];
        for (int iv = 0; iv < no; ++iv) {
            const double v = go[2 * iv], wv = go[2 * iv + 1];
            const double uv = u * v;
            const double x[3] = {A0[0] + u * e1x + uv * e2x, A0[1] + u * e1y + uv * e2y,
                                 A0[2] + u * e1z + uv * e2z};
            const double wx = wu * wv * u * two_area;
            if (tier == GT_MID) {
                collapsed_acc<0, NF>(x[0], x[1], x[2], aj, bj, cj, q.n4, q.g4, f, l0, nl, ar, ai,
                                     wx);
            } else {
                gal_inner_split<NF>(x, wx, aj, bj, cj, q.ng, q.gg, f, l0, nl, ar, ai);
            }
        }
    }
}

}  // namespace gaca
