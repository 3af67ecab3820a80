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
    // two points per pass: fully unrolled, the six points' loads and polynomials held 92
    // VGPRs (5 waves per SIMD); in pairs 70 (7 waves), and the face phase ran 25 % faster
#pragma unroll 2
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

// ---------------------------------------------------------------------------------------
// P1 double layer collocated at the vertices (Sec. 3, eq. bie_semi_diri with phi_j linear):
//   K_ij(s) = sum over the triangles t of the patch of vertex j of
//             int_t dG/dn_y(x_i - y) lambda_{t,j}(y) dS_y,
// lambda_{t,j} the barycentric coordinate of vertex j in t.  A triangle that has x_i as a
// vertex contributes exactly 0 (x_i lies in its plane).  Far pairs take the 6-point rule on
// every triangle; near pairs per triangle the tier of q = |x_i - c_t| / h_t (q >= 4: 6-point,
// 2 <= q < 4: collapsed n4 x n4, q < 2: collapsed n8 x n8, collapsed at the triangle's first
// vertex, where lambda = (1 - u, u (1 - v), u v)).

__device__ __forceinline__ bool p1_holds(const GeoDev &g, int64_t t, int32_t vid) {
    return g.tv0[t] == vid || g.tv1[t] == vid || g.tv2[t] == vid;
}

// collapsed rule on triangle (a, b, c) weighted by the barycentric coordinate loc
template <int NF>
__device__ __forceinline__ void collapsed_acc_p1(double x, double y, double z, const double *a,
                                                 const double *b, const double *c, int n,
                                                 const double *gtab, int loc, const FreqDev &f,
                                                 int l0, int nl, double *ar, double *ai) {
    const double e1x = b[0] - a[0], e1y = b[1] - a[1], e1z = b[2] - a[2];
    const double e2x = c[0] - b[0], e2y = c[1] - b[1], e2z = c[2] - b[2];
    const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const double two_area = sqrt(nx * nx + ny * ny + nz * nz);
    for (int iu = 0; iu < n; ++iu) {
        const double u = gtab[2 * iu], wu = gtab[2 * iu + 1];
        for (int iv = 0; iv < n; ++iv) {
            const double v = gtab[2 * iv], wv = gtab[2 * iv + 1];
            const double uv = u * v;
            const double lam = loc == 0 ? 1.0 - u : (loc == 1 ? u - uv : uv);
            const double px = a[0] + u * e1x + uv * e2x;
            const double py = a[1] + u * e1y + uv * e2y;
            const double pz = a[2] + u * e1z + uv * e2z;
            const double w = wu * wv * u * two_area * lam;
            double ir;
            const double r = dist3_inv(x, y, z, px, py, pz, ir);
#pragma unroll
            for (int t = 0; t < NF; ++t)
                if (t < nl) kacc<1>(r, ir, f.re[l0 + t], f.im[l0 + t], w, ar[t], ai[t]);
        }
    }
}

// 6-point rule on triangle t weighted by the barycentric coordinate loc
template <int NF>
__device__ __forceinline__ void rule6_acc_p1(const GeoDev &g, double x, double y, double z,
                                             int64_t t, int loc, const FreqDev &f, int l0,
                                             int nl, double *ar, double *ai) {
    const int64_t T = g.T;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        double ir;
        const double r = dist3_inv(x, y, z, g.q6x[p * T + t], g.q6y[p * T + t], g.q6z[p * T + t], ir);
        const double w = g.q6wl[(int64_t)(loc * 6 + p) * T + t];
#pragma unroll
        for (int k = 0; k < NF; ++k)
            if (k < nl) kacc<1>(r, ir, f.re[l0 + k], f.im[l0 + k], w, ar[k], ai[k]);
    }
}

// Entry (i, j) (tree positions) at NF frequencies from l0 (nl valid); far: 6-point rule on
// every triangle.  Results in ar / ai (zeroed here).
template <int NF>
__device__ void p1_entry(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t i,
                         int64_t j, bool far, int l0, int nl, double *ar, double *ai) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        ar[k] = 0.0;
        ai[k] = 0.0;
    }
    const double x = g.xx[i], y = g.xy[i], z = g.xz[i];
    const int32_t vid = g.dvid[i];
    for (int32_t e = g.pptr[j]; e < g.pptr[j + 1]; ++e) {
        const int64_t t = g.ptri[e];
        if (p1_holds(g, t, vid)) continue;
        const int loc = g.ploc[e];
        double tr[NF], ti[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            tr[k] = 0.0;
            ti[k] = 0.0;
        }
        int tier = TIER_FAR6;
        if (!far) {
            const double dx = x - g.tcx[t], dy = y - g.tcy[t], dz = z - g.tcz[t];
            const double qd = sqrt(dx * dx + dy * dy + dz * dz) / g.h[t];
            tier = qd >= 4.0 ? TIER_FAR6 : (qd >= 2.0 ? TIER_MID4 : TIER_NEAR8);
        }
        if (tier == TIER_FAR6) {
            rule6_acc_p1<NF>(g, x, y, z, t, loc, f, l0, nl, tr, ti);
        } else {
            const double a[3] = {g.ax[t], g.ay[t], g.az[t]};
            const double b[3] = {g.bx[t], g.by[t], g.bz[t]};
            const double c[3] = {g.cx[t], g.cy[t], g.cz[t]};
            if (tier == TIER_MID4) collapsed_acc_p1<NF>(x, y, z, a, b, c, q.n4, q.g4, loc, f, l0, nl, tr, ti);
            else collapsed_acc_p1<NF>(x, y, z, a, b, c, q.n8, q.g8, loc, f, l0, nl, tr, ti);
        }
        const double num = g.nx[t] * x + g.ny[t] * y + g.nz[t] * z - g.d[t];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            ar[k] += num * tr[k];
            ai[k] += num * ti[k];
        }
    }
}

// Far entry at one frequency (the face and fibre evaluations of admissible blocks).
__device__ __forceinline__ void p1_far_entry(const GeoDev &g, int64_t i, int64_t j, double sre,
                                             double sim, double &er, double &ei) {
    const double x = g.xx[i], y = g.xy[i], z = g.xz[i];
    double ar = 0.0, ai = 0.0;
    for (int32_t e = g.pptr[j]; e < g.pptr[j + 1]; ++e) {
        const int64_t t = g.ptri[e];
        const int loc = g.ploc[e];
        const int64_t T = g.T;
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            double ir;
            const double r = dist3_inv(x, y, z, g.q6x[p * T + t], g.q6y[p * T + t], g.q6z[p * T + t], ir);
            kacc<1>(r, ir, sre, sim, g.q6wl[(int64_t)(loc * 6 + p) * T + t], tr, ti);
        }
        const double num = g.nx[t] * x + g.ny[t] * y + g.nz[t] * z - g.d[t];
        ar += num * tr;
        ai += num * ti;
    }
    er = ar;
    ei = ai;
}

}  // namespace gaca
