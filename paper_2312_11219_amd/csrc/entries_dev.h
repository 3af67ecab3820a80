// Device-side evaluation of the integrated Laplace-domain kernels (Sec. 3 of the paper):
//   single layer  G_s(r)   = exp(-s r) / (4 pi r)
//   double layer  dG/dn_y  = exp(-s r) (1 + s r) ((x - y) . n_y) / (4 pi r^3),
// with (x - y) . n_j = n_j . x - d_j for y in the plane of triangle j (exactly 0 for
// coplanar pairs).  Collocation entries integrate over triangle j at the centroid x_i:
//   far blocks and q >= 4:   6-point symmetric degree-4 rule
//   2 <= q < 4:              collapsed (Duffy square) Gauss 4 x 4
//   q < 2, i != j:           collapsed Gauss 8 x 8
//   i == j:                  three Duffy sub-triangles split at x_i, n_D x n_D
// where q = |x_i - x_j| / h_j.  The double layer self entry is 0.
#pragma once

#include "fastmath_dev.h"
#include "internal.h"

namespace gaca {

constexpr double kFourPi = 12.566370614359172953850573533118;  // 4 pi

constexpr double kInvFourPi = 0.079577471545947667884441881686257181;  // 1 / (4 pi)

// Accumulate w * G(s, r) (SLP) or w * exp(-s r)(1 + s r)/(4 pi r^3) (DLP, numerator applied
// by the caller) into (ar, ai); ir = 1 / r.
template <int KERNEL>
__device__ __forceinline__ void kacc(double r, double ir, double sre, double sim, double w,
                                     double &ar, double &ai) {
    double mag = fm::exp(-sre * r);
    double sn, cs;
    fm::sincos(sim * r, &sn, &cs);
    double er = mag * cs, ei = -mag * sn;
    if (KERNEL == 0) {
        double c = w * kInvFourPi * ir;
        ar += c * er;
        ai += c * ei;
    } else {
        double fr = 1.0 + sre * r, fi = sim * r;
        double c = w * kInvFourPi * (ir * ir * ir);
        ar += c * (er * fr - ei * fi);
        ai += c * (er * fi + ei * fr);
    }
}

__device__ __forceinline__ double dist3(double x, double y, double z, double px, double py,
                                        double pz) {
    double dx = x - px, dy = y - py, dz = z - pz;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// r = |x - p| and ir = 1 / r from one reciprocal square root: the hardware estimate of
// d^-1/2 refined by two Newton-Raphson steps t <- t + t (1 - d t^2) / 2 (each roughly
// doubles the correct bits), then r = d t.
__device__ __forceinline__ double dist3_inv(double x, double y, double z, double px, double py,
                                            double pz, double &ir) {
    const double dx = x - px, dy = y - py, dz = z - pz;
    const double d = dx * dx + dy * dy + dz * dz;
    double t = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-d * t, t, 1.0);
        t = fma(0.5 * t, e, t);
    }
    ir = t;
    return d * t;
}

// Far rule entry at one frequency for collocation point x (row element i) and element j.
template <int KERNEL>
__device__ __forceinline__ void entry_far6(const GeoDev &g, double x, double y, double z,
                                           int64_t j, double sre, double sim, double &er,
                                           double &ei) {
    double ar = 0.0, ai = 0.0;
    const int64_t M = g.M;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        double ir;
        double r = dist3_inv(x, y, z, g.q6x[p * M + j], g.q6y[p * M + j], g.q6z[p * M + j], ir);
        kacc<KERNEL>(r, ir, sre, sim, g.q6w[p * M + j], ar, ai);
    }
    if (KERNEL == 1) {
        double num = g.nx[j] * x + g.ny[j] * y + g.nz[j] * z - g.d[j];
        ar *= num;
        ai *= num;
    }
    er = ar;
    ei = ai;
}

// Mixed-precision far entry divided by the block scale c = exp(-s d0), FP32 arithmetic:
//   sum_q w_q exp(-s (r_q - d0)) / (4 pi r_q)         (SLP)
//   num * sum_q w_q exp(-s (r_q - d0)) (1 + s r_q) / (4 pi r_q^3)   (DLP)
// with D = x_sigma - y_tau (box centres, d0 = |D|), a = (x_i - x_sigma) - (y_q - y_tau) and
// r - d0 = (2 a.D + a.a) / (r + d0), free of cancellation; the exponent stays within
// +-Re(s) (radius_sigma + radius_tau) so FP32 neither over- nor underflows.
template <int KERNEL>
__device__ __forceinline__ float2 entry_far6_scaled(const GeoDev &g, float ax, float ay,
                                                    float az, float Dx, float Dy, float Dz,
                                                    float d0, float kappa, int64_t j, float cjx,
                                                    float cjy, float cjz, float sre, float sim,
                                                    float num) {
    float ar = 0.0f, ai = 0.0f;
    const int64_t M = g.M;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const float bx = cjx + g.q6dx[p * M + j], by = cjy + g.q6dy[p * M + j],
                    bz = cjz + g.q6dz[p * M + j];
        const float qx = ax - bx, qy = ay - by, qz = az - bz;
        const float vx = qx + Dx, vy = qy + Dy, vz = qz + Dz;
        const float r = sqrtf(vx * vx + vy * vy + vz * vz);
        const float dr =
            (2.0f * (qx * Dx + qy * Dy + qz * Dz) + (qx * qx + qy * qy + qz * qz) + kappa) / (r + d0);
        const float mag = expf(-sre * dr);
        float sn, cs;
        sincosf(sim * dr, &sn, &cs);
        const float er = mag * cs, ei = -mag * sn;
        const float w = g.q6wf[p * M + j];
        if (KERNEL == 0) {
            const float c = w / (12.566370614359172f * r);
            ar += c * er;
            ai += c * ei;
        } else {
            const float fr = 1.0f + sre * r, fi = sim * r;
            const float c = w / (12.566370614359172f * r * r * r);
            ar += c * (er * fr - ei * fi);
            ai += c * (er * fi + ei * fr);
        }
    }
    if (KERNEL == 1) {
        ar *= num;
        ai *= num;
    }
    return make_float2(ar, ai);
}

// Tier of a collocation pair inside a near block (host computes the same with the same
// operations; the device version is used only by the test hook).
__device__ __forceinline__ int tier_of(const GeoDev &g, int64_t i, int64_t j) {
    if (i == j) return TIER_SELF;
    double q = dist3(g.xx[i], g.xy[i], g.xz[i], g.xx[j], g.xy[j], g.xz[j]) / g.h[j];
    return q >= 4.0 ? TIER_FAR6 : (q >= 2.0 ? TIER_MID4 : TIER_NEAR8);
}

// Collapsed n x n rule on triangle (a, b, c) collapsed at a: y = a + u (b - a) + u v (c - b),
// weight wu wv u |(b - a) x (c - b)|; accumulates NF frequencies starting at l0.
template <int KERNEL, int NF>
__device__ __forceinline__ void collapsed_acc(double x, double y, double z, const double *a,
                                             const double *b, const double *c, int n,
                                             const double *gtab, const FreqDev &f, int l0,
                                             int nl, double *ar, double *ai,
                                             double wscale = 1.0) {
    double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    double e2x = c[0] - b[0], e2y = c[1] - b[1], e2z = c[2] - b[2];
    double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    double two_area = sqrt(nx * nx + ny * ny + nz * nz);
    for (int iu = 0; iu < n; ++iu) {
        double u = gtab[2 * iu], wu = gtab[2 * iu + 1];
        for (int iv = 0; iv < n; ++iv) {
            double v = gtab[2 * iv], wv = gtab[2 * iv + 1];
            double uv = u * v;
            double px = a[0] + u * e1x + uv * e2x;
            double py = a[1] + u * e1y + uv * e2y;
            double pz = a[2] + u * e1z + uv * e2z;
            double w = wu * wv * u * two_area * wscale;
            double ir;
            double r = dist3_inv(x, y, z, px, py, pz, ir);
#pragma unroll
            for (int t = 0; t < NF; ++t)
                if (t < nl) kacc<KERNEL>(r, ir, f.re[l0 + t], f.im[l0 + t], w, ar[t], ai[t]);
        }
    }
}

// Near-block collocation entry of pair (i, j) with the given tier at NF frequencies
// starting at l0 (nl <= NF valid).  Results in ar/ai (zeroed here).
template <int KERNEL, int NF>
__device__ void near_entry(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t i,
                           int64_t j, int tier, int l0, int nl, double *ar, double *ai) {
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        ar[t] = 0.0;
        ai[t] = 0.0;
    }
    if (tier == TIER_SELF && KERNEL == 1) return;
    const double x = g.xx[i], y = g.xy[i], z = g.xz[i];
    const double a[3] = {g.ax[j], g.ay[j], g.az[j]};
    const double b[3] = {g.bx[j], g.by[j], g.bz[j]};
    const double c[3] = {g.cx[j], g.cy[j], g.cz[j]};
    if (tier == TIER_FAR6) {
        const int64_t M = g.M;
        for (int p = 0; p < 6; ++p) {
            double ir;
            double r = dist3_inv(x, y, z, g.q6x[p * M + j], g.q6y[p * M + j], g.q6z[p * M + j], ir);
            double w = g.q6w[p * M + j];
#pragma unroll
            for (int t = 0; t < NF; ++t)
                if (t < nl) kacc<KERNEL>(r, ir, f.re[l0 + t], f.im[l0 + t], w, ar[t], ai[t]);
        }
    } else if (tier == TIER_MID4) {
        collapsed_acc<KERNEL, NF>(x, y, z, a, b, c, q.n4, q.g4, f, l0, nl, ar, ai);
    } else if (tier == TIER_NEAR8) {
        collapsed_acc<KERNEL, NF>(x, y, z, a, b, c, q.n8, q.g8, f, l0, nl, ar, ai);
    } else {
        const double xc[3] = {x, y, z};
        collapsed_acc<KERNEL, NF>(x, y, z, xc, b, c, q.nd, q.gd, f, l0, nl, ar, ai);
        collapsed_acc<KERNEL, NF>(x, y, z, xc, c, a, q.nd, q.gd, f, l0, nl, ar, ai);
        collapsed_acc<KERNEL, NF>(x, y, z, xc, a, b, q.nd, q.gd, f, l0, nl, ar, ai);
    }
    if (KERNEL == 1) {
        double num = g.nx[j] * x + g.ny[j] * y + g.nz[j] * z - g.d[j];
#pragma unroll
        for (int t = 0; t < NF; ++t) {
            ar[t] *= num;
            ai[t] *= num;
        }
    }
}

}  // namespace gaca
