// Galerkin operators of the Neumann problem with linear continuous test and trial functions
// (Sec. 3, eq. bie_semi_neum), on the device:
//   hypersingular D_ij = sum over triangle pairs (t in supp phi_i, t' in supp phi_j) of
//       (curl l_a . curl l_b) int int G + s^2 (n_t . n_t') int int G l_a(x) l_b(y),
//     the form after integration by parts (wave number k = i s of the Helmholtz analogue);
//   adjoint double layer K'_ij = sum over the same pairs of int int dG/dn_x l_a(x) l_b(y),
//     dG/dn_x = -((x - y) . n_x) e^{-s r} (1 + s r) / (4 pi r^3),
// l_a, l_b the barycentric coordinates of vertex i in t and of vertex j in t' (the hat
// functions on those triangles), curl l_a = -e_a / (2 A) (e_a the edge opposite to a).
// Triangle pairs: far blocks and disjoint pairs with q >= 4 take 6 x 6 points; 2 <= q < 4
// collapsed n4 x n4 on both; q < 2 an outer collapsed ng x ng rule on t and the inner
// integral over t' split at the point of t' nearest to the outer point into three Duffy
// triangles; identical, edge- and vertex-sharing pairs the Sauter-Schwab maps of [0,1]^4
// (6, 5, 2 regions) with ns points per variable.  q = |c_t - c_t'| / max(h_t, h_t').  The
// dG/dn_x integrand of a coplanar pair is 0.  Geometry: the P1 layout of GeoDev.
#pragma once

#include "entries_dev.h"

namespace gaca {

// kernel value without weight: OP 0 G_s = e^{-s r} / (4 pi r); OP 1 e^{-s r} (1 + s r) /
// (4 pi r^3) (the numerator of dG/dn_x is applied by the caller)
template <int OP>
__device__ __forceinline__ void gp1_kval(double r, double ir, double sre, double sim, double &gr,
                                         double &gi) {
    const double mag = fm::exp(-sre * r);
    double sn, cs;
    fm::sincos(sim * r, &sn, &cs);
    const double er = mag * cs, ei = -mag * sn;
    if (OP == 0) {
        const double c = kInvFourPi * ir;
        gr = c * er;
        gi = c * ei;
    } else {
        const double fr = 1.0 + sre * r, fi = sim * r;
        const double c = kInvFourPi * ir * ir * ir;
        gr = c * (er * fr - ei * fi);
        gi = c * (er * fi + ei * fr);
    }
}

// accumulators of one triangle pair: S = int int k (OP 0 only), M = int int k l_a l_b
template <int NF>
struct GP1Acc {
    double sr[NF], si[NF], mr[NF], mi[NF];
};

// one point pair (x, y), weight w, la = l_a(x), lb = l_b(y)
template <int OP, int NF>
__device__ __forceinline__ void gp1_add(const double *x, double la, const double *y, double lb,
                                        double w, const double *nx, const FreqDev &f, int l0,
                                        int nl, GP1Acc<NF> &A) {
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    const double d = dx * dx + dy * dy + dz * dz;
    double t = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) t = fma(0.5 * t, fma(-d * t, t, 1.0), t);
    const double r = d * t;
    const double num = OP == 1 ? -(dx * nx[0] + dy * nx[1] + dz * nx[2]) : 1.0;
    const double wm = w * la * lb * num;
#pragma unroll
    for (int k = 0; k < NF; ++k)
        if (k < nl) {
            double gr, gi;
            gp1_kval<OP>(r, t, f.re[l0 + k], f.im[l0 + k], gr, gi);
            if (OP == 0) {
                A.sr[k] += w * gr;
                A.si[k] += w * gi;
            }
            A.mr[k] += wm * gr;
            A.mi[k] += wm * gi;
        }
}

struct GP1Tri {
    double v[3][3];
    double n[3], c[3];
    double area, h;
};

__device__ __forceinline__ void gp1_load(const GeoDev &g, int64_t t, GP1Tri &T) {
    T.v[0][0] = g.ax[t]; T.v[0][1] = g.ay[t]; T.v[0][2] = g.az[t];
    T.v[1][0] = g.bx[t]; T.v[1][1] = g.by[t]; T.v[1][2] = g.bz[t];
    T.v[2][0] = g.cx[t]; T.v[2][1] = g.cy[t]; T.v[2][2] = g.cz[t];
    T.n[0] = g.nx[t]; T.n[1] = g.ny[t]; T.n[2] = g.nz[t];
    T.c[0] = g.tcx[t]; T.c[1] = g.tcy[t]; T.c[2] = g.tcz[t];
    T.area = g.area[t];
    T.h = g.h[t];
}

// barycentric coordinate `a` of y (a point of T's plane)
__device__ __forceinline__ double gp1_bary(const GP1Tri &T, const double *y, int a) {
    double e1[3], e2[3], d[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = T.v[1][k] - T.v[0][k];
        e2[k] = T.v[2][k] - T.v[0][k];
        d[k] = y[k] - T.v[0][k];
    }
    const double A = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const double B = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const double C = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const double p = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
    const double q = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
    const double det = A * C - B * B;
    const double u = (C * p - B * q) / det, v = (A * q - B * p) / det;
    return a == 0 ? 1.0 - u - v : (a == 1 ? u : v);
}

// collapsed rule point (u, v) on (a, b, c) collapsed at a: position and weight (measure)
__device__ __forceinline__ void gp1_collapsed_pt(const double *a, const double *b, const double *c,
                                                 double u, double v, double wuv, double *y,
                                                 double &w) {
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - b[k];
    }
    const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                 nz = e1[0] * e2[1] - e1[1] * e2[0];
    for (int k = 0; k < 3; ++k) y[k] = a[k] + u * e1[k] + u * v * e2[k];
    w = wuv * u * sqrt(nx * nx + ny * ny + nz * nz);
}

// closest point of triangle (a, b, c) to x
__device__ void gp1_closest(const double *x, const double *a, const double *b, const double *c,
                            double *p) {
    double ab[3], ac[3], ap[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ap[k] = x[k] - a[k];
    }
    auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int k = 0; k < 3; ++k) p[k] = a[k];
        return;
    }
    double bp[3];
    for (int k = 0; k < 3; ++k) bp[k] = x[k] - b[k];
    const double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) {
        for (int k = 0; k < 3; ++k) p[k] = b[k];
        return;
    }
    const double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + v * ab[k];
        return;
    }
    double cp[3];
    for (int k = 0; k < 3; ++k) cp[k] = x[k] - c[k];
    const double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) {
        for (int k = 0; k < 3; ++k) p[k] = c[k];
        return;
    }
    const double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        const double w = d2 / (d2 - d6);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + w * ac[k];
        return;
    }
    const double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int k = 0; k < 3; ++k) p[k] = b[k] + w * (c[k] - b[k]);
        return;
    }
    const double den = 1.0 / (va + vb + vc);
    const double v = vb * den, w = vc * den;
    for (int k = 0; k < 3; ++k) p[k] = a[k] + ab[k] * v + ac[k] * w;
}

// regularising maps: region r of relation rel (3 identical, 2 edge, 1 vertex) at
// (xi, e1, e2, e3): reference points X, Y of the two triangles and the Jacobian factor
__device__ __forceinline__ void gp1_ss_region(int rel, int r, double xi, double e1, double e2,
                                              double e3, double *X, double *Y, double &jac) {
    if (rel == 3) {
        jac = xi * xi * xi * e1 * e1 * e2;
        const int pr = r >> 1;
        double a1, a2, b1, b2;
        if (pr == 0) {
            a1 = xi; a2 = xi * (1.0 - e1 + e1 * e2);
            b1 = xi * (1.0 - e1 * e2 * e3); b2 = xi * (1.0 - e1);
        } else if (pr == 1) {
            a1 = xi; a2 = xi * e1 * (1.0 - e2 + e2 * e3);
            b1 = xi * (1.0 - e1 * e2); b2 = xi * e1 * (1.0 - e2);
        } else {
            a1 = xi * (1.0 - e1 * e2 * e3); a2 = xi * e1 * (1.0 - e2 * e3);
            b1 = xi; b2 = xi * e1 * (1.0 - e2);
        }
        // regions come in pairs with the roles of the two points exchanged
        if ((r & 1) == 0) {
            X[0] = a1; X[1] = a2; Y[0] = b1; Y[1] = b2;
        } else {
            X[0] = b1; X[1] = b2; Y[0] = a1; Y[1] = a2;
        }
    } else if (rel == 2) {
        jac = xi * xi * xi * e1 * e1 * (r == 0 ? 1.0 : e2);
        if (r == 0) {
            X[0] = xi; X[1] = xi * e1 * e3;
            Y[0] = xi * (1.0 - e1 * e2); Y[1] = xi * e1 * (1.0 - e2);
        } else if (r == 1) {
            X[0] = xi; X[1] = xi * e1;
            Y[0] = xi * (1.0 - e1 * e2 * e3); Y[1] = xi * e1 * e2 * (1.0 - e3);
        } else if (r == 2) {
            X[0] = xi * (1.0 - e1 * e2); X[1] = xi * e1 * (1.0 - e2);
            Y[0] = xi; Y[1] = xi * e1 * e2 * e3;
        } else if (r == 3) {
            X[0] = xi * (1.0 - e1 * e2 * e3); X[1] = xi * e1 * e2 * (1.0 - e3);
            Y[0] = xi; Y[1] = xi * e1;
        } else {
            X[0] = xi * (1.0 - e1 * e2 * e3); X[1] = xi * e1 * (1.0 - e2 * e3);
            Y[0] = xi; Y[1] = xi * e1 * e2;
        }
    } else {
        jac = xi * xi * xi * e2;
        if (r == 0) {
            X[0] = xi; X[1] = xi * e1;
            Y[0] = xi * e2; Y[1] = xi * e2 * e3;
        } else {
            X[0] = xi * e2; X[1] = xi * e2 * e1;
            Y[0] = xi; Y[1] = xi * e3;
        }
    }
}

// Local integrals of the triangle pair (ti, tj) for vertex a of ti and b of tj (original
// local indices), NF frequencies from l0; accumulates into A (zeroed by the caller).
template <int OP, int NF>
__device__ void gp1_pair(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t ti, int a,
                         int64_t tj, int b, bool far, int l0, int nl, GP1Acc<NF> &A) {
    GP1Tri Ti, Tj;
    gp1_load(g, ti, Ti);
    gp1_load(g, tj, Tj);
    if (OP == 1) {   // coplanar: (x - y) . n_x = 0 on tj
        bool cop = true;
        for (int c = 0; c < 3; ++c) {
            const double dd = (Tj.v[c][0] - Ti.v[0][0]) * Ti.n[0] + (Tj.v[c][1] - Ti.v[0][1]) * Ti.n[1] +
                              (Tj.v[c][2] - Ti.v[0][2]) * Ti.n[2];
            if (fabs(dd) > 1e-14 * Ti.h) cop = false;
        }
        if (cop) return;
    }
    const int32_t vi[3] = {g.tv0[ti], g.tv1[ti], g.tv2[ti]};
    const int32_t vj[3] = {g.tv0[tj], g.tv1[tj], g.tv2[tj]};
    int shared = 0, si[3] = {0, 0, 0}, sj[3] = {0, 0, 0};
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y)
            if (vi[x] == vj[y]) {
                si[shared] = x;
                sj[shared] = y;
                ++shared;
            }
    if (shared > 0) {
        // reordered vertices: identical the triangle's own order; edge the shared vertices
        // in ti's order then the third; vertex each list rotated to start at the shared one
        int pa[3], pb[3];
        if (shared == 3) {
            for (int c = 0; c < 3; ++c) pa[c] = pb[c] = c;
        } else if (shared == 2) {
            const int a0 = si[0] < si[1] ? 0 : 1, a1 = 1 - a0;
            pa[0] = si[a0]; pa[1] = si[a1]; pa[2] = 3 - si[0] - si[1];
            pb[0] = sj[a0]; pb[1] = sj[a1]; pb[2] = 3 - sj[0] - sj[1];
        } else {
            for (int c = 0; c < 3; ++c) {
                pa[c] = (si[0] + c) % 3;
                pb[c] = (sj[0] + c) % 3;
            }
        }
        // reordered index of the selected vertices (lambda of reordered vertex c)
        int ra = 0, rb = 0;
        for (int c = 0; c < 3; ++c) {
            if (pa[c] == a) ra = c;
            if (pb[c] == b) rb = c;
        }
        const double *P0 = Ti.v[pa[0]], *P1 = Ti.v[pa[1]], *P2 = Ti.v[pa[2]];
        const double *Q0 = Tj.v[pb[0]], *Q1 = Tj.v[pb[1]], *Q2 = Tj.v[pb[2]];
        const double jij = 4.0 * Ti.area * Tj.area;
        const int nreg = shared == 3 ? 6 : (shared == 2 ? 5 : 2);
        const int n = q.ns;
        for (int i1 = 0; i1 < n; ++i1)
            for (int i2 = 0; i2 < n; ++i2)
                for (int i3 = 0; i3 < n; ++i3)
                    for (int i4 = 0; i4 < n; ++i4) {
                        const double xi = q.gs[2 * i1], e1 = q.gs[2 * i2], e2 = q.gs[2 * i3],
                                     e3 = q.gs[2 * i4];
                        const double w0 = q.gs[2 * i1 + 1] * q.gs[2 * i2 + 1] * q.gs[2 * i3 + 1] *
                                          q.gs[2 * i4 + 1] * jij;
                        for (int r = 0; r < nreg; ++r) {
                            double X[2], Y[2], jac;
                            gp1_ss_region(shared, r, xi, e1, e2, e3, X, Y, jac);
                            double x[3], y[3];
                            for (int k = 0; k < 3; ++k) {
                                x[k] = P0[k] + X[0] * (P1[k] - P0[k]) + X[1] * (P2[k] - P1[k]);
                                y[k] = Q0[k] + Y[0] * (Q1[k] - Q0[k]) + Y[1] * (Q2[k] - Q1[k]);
                            }
                            const double la = ra == 0 ? 1.0 - X[0] : (ra == 1 ? X[0] - X[1] : X[1]);
                            const double lb = rb == 0 ? 1.0 - Y[0] : (rb == 1 ? Y[0] - Y[1] : Y[1]);
                            gp1_add<OP, NF>(x, la, y, lb, w0 * jac, Ti.n, f, l0, nl, A);
                        }
                    }
        return;
    }
    const double dcx = Ti.c[0] - Tj.c[0], dcy = Ti.c[1] - Tj.c[1], dcz = Ti.c[2] - Tj.c[2];
    const double qd = sqrt(dcx * dcx + dcy * dcy + dcz * dcz) / fmax(Ti.h, Tj.h);
    if (far || qd >= 4.0) {
        const int64_t T = g.T;
        for (int p = 0; p < 6; ++p) {
            const double x[3] = {g.q6x[p * T + ti], g.q6y[p * T + ti], g.q6z[p * T + ti]};
            // weight x area x lambda: the plain weight is the sum over the three lambdas
            const double wa0 = g.q6wl[(int64_t)(0 * 6 + p) * T + ti], wa1 = g.q6wl[(int64_t)(6 + p) * T + ti],
                         wa2 = g.q6wl[(int64_t)(12 + p) * T + ti];
            const double wx = wa0 + wa1 + wa2;
            const double la = (a == 0 ? wa0 : (a == 1 ? wa1 : wa2)) / wx;
            for (int p2 = 0; p2 < 6; ++p2) {
                const double y[3] = {g.q6x[p2 * T + tj], g.q6y[p2 * T + tj], g.q6z[p2 * T + tj]};
                const double wb0 = g.q6wl[(int64_t)(0 * 6 + p2) * T + tj], wb1 = g.q6wl[(int64_t)(6 + p2) * T + tj],
                             wb2 = g.q6wl[(int64_t)(12 + p2) * T + tj];
                const double wy = wb0 + wb1 + wb2;
                const double lb = (b == 0 ? wb0 : (b == 1 ? wb1 : wb2)) / wy;
                gp1_add<OP, NF>(x, la, y, lb, wx * wy, Ti.n, f, l0, nl, A);
            }
        }
        return;
    }
    if (qd >= 2.0) {
        const int n = q.n4;
        for (int iu = 0; iu < n; ++iu)
            for (int iv = 0; iv < n; ++iv) {
                const double u = q.g4[2 * iu], v = q.g4[2 * iv];
                double x[3], wx;
                gp1_collapsed_pt(Ti.v[0], Ti.v[1], Ti.v[2], u, v, q.g4[2 * iu + 1] * q.g4[2 * iv + 1], x, wx);
                const double la = a == 0 ? 1.0 - u : (a == 1 ? u - u * v : u * v);
                for (int ju = 0; ju < n; ++ju)
                    for (int jv = 0; jv < n; ++jv) {
                        const double u2 = q.g4[2 * ju], v2 = q.g4[2 * jv];
                        double y[3], wy;
                        gp1_collapsed_pt(Tj.v[0], Tj.v[1], Tj.v[2], u2, v2, q.g4[2 * ju + 1] * q.g4[2 * jv + 1], y, wy);
                        const double lb = b == 0 ? 1.0 - u2 : (b == 1 ? u2 - u2 * v2 : u2 * v2);
                        gp1_add<OP, NF>(x, la, y, lb, wx * wy, Ti.n, f, l0, nl, A);
                    }
            }
        return;
    }
    const int n = q.ng;
    for (int iu = 0; iu < n; ++iu)
        for (int iv = 0; iv < n; ++iv) {
            const double u = q.gg[2 * iu], v = q.gg[2 * iv];
            double x[3], wx;
            gp1_collapsed_pt(Ti.v[0], Ti.v[1], Ti.v[2], u, v, q.gg[2 * iu + 1] * q.gg[2 * iv + 1], x, wx);
            const double la = a == 0 ? 1.0 - u : (a == 1 ? u - u * v : u * v);
            double cp[3];
            gp1_closest(x, Tj.v[0], Tj.v[1], Tj.v[2], cp);
            for (int piece = 0; piece < 3; ++piece) {
                const double *pb_ = Tj.v[(piece + 1) % 3], *pc_ = Tj.v[(piece + 2) % 3];
                for (int ju = 0; ju < n; ++ju)
                    for (int jv = 0; jv < n; ++jv) {
                        double y[3], wy;
                        gp1_collapsed_pt(cp, pb_, pc_, q.gg[2 * ju], q.gg[2 * jv],
                                         q.gg[2 * ju + 1] * q.gg[2 * jv + 1], y, wy);
                        const double lb = gp1_bary(Tj, y, b);
                        gp1_add<OP, NF>(x, la, y, lb, wx * wy, Ti.n, f, l0, nl, A);
                    }
            }
        }
}

// curl of l_a on T: -(v[a+2] - v[a+1]) / (2 A)
__device__ __forceinline__ void gp1_curl(const GeoDev &g, int64_t t, int a, double *c) {
    const double vx[3] = {g.ax[t], g.bx[t], g.cx[t]}, vy[3] = {g.ay[t], g.by[t], g.cy[t]},
                 vz[3] = {g.az[t], g.bz[t], g.cz[t]};
    const int b = (a + 1) % 3, d = (a + 2) % 3;
    const double s = -0.5 / g.area[t];
    c[0] = s * (vx[d] - vx[b]);
    c[1] = s * (vy[d] - vy[b]);
    c[2] = s * (vz[d] - vz[b]);
}

// Entry (i, j) (tree positions) of operator OP (0 hypersingular, 1 adjoint double layer) at
// NF frequencies from l0; results in ar / ai (zeroed here).
template <int OP, int NF>
__device__ void gp1_entry(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t i,
                          int64_t j, bool far, int l0, int nl, double *ar, double *ai) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        ar[k] = 0.0;
        ai[k] = 0.0;
    }
    for (int32_t e = g.pptr[i]; e < g.pptr[i + 1]; ++e) {
        const int64_t ti = g.ptri[e];
        const int a = g.ploc[e];
        for (int32_t e2 = g.pptr[j]; e2 < g.pptr[j + 1]; ++e2) {
            const int64_t tj = g.ptri[e2];
            const int b = g.ploc[e2];
            GP1Acc<NF> A;
#pragma unroll
            for (int k = 0; k < NF; ++k) A.sr[k] = A.si[k] = A.mr[k] = A.mi[k] = 0.0;
            gp1_pair<OP, NF>(g, q, f, ti, a, tj, b, far, l0, nl, A);
            if (OP == 1) {
#pragma unroll
                for (int k = 0; k < NF; ++k) {
                    ar[k] += A.mr[k];
                    ai[k] += A.mi[k];
                }
            } else {
                double ca[3], cb[3];
                gp1_curl(g, ti, a, ca);
                gp1_curl(g, tj, b, cb);
                const double cc = ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2];
                const double nn = g.nx[ti] * g.nx[tj] + g.ny[ti] * g.ny[tj] + g.nz[ti] * g.nz[tj];
#pragma unroll
                for (int k = 0; k < NF; ++k)
                    if (k < nl) {
                        const double sr = f.re[l0 + k], si = f.im[l0 + k];
                        const double s2r = sr * sr - si * si, s2i = 2.0 * sr * si;
                        const double tr = nn * (s2r * A.mr[k] - s2i * A.mi[k]);
                        const double ti2 = nn * (s2r * A.mi[k] + s2i * A.mr[k]);
                        ar[k] += cc * A.sr[k] + tr;
                        ai[k] += cc * A.si[k] + ti2;
                    }
            }
        }
    }
}

// Far entry at one frequency (face and fibre evaluations of admissible blocks: 6 x 6 points
// on every triangle pair).
template <int OP>
__device__ __forceinline__ void gp1_far_entry(const GeoDev &g, const QuadDev &q, int64_t i,
                                              int64_t j, const double *sre, const double *sim,
                                              int k, double &er, double &ei) {
    FreqDev f1{};
    f1.re = sre;
    f1.im = sim;
    double ar[1], ai[1];
    gp1_entry<OP, 1>(g, q, f1, i, j, true, k, 1, ar, ai);
    er = ar[0];
    ei = ai[0];
}

}  // namespace gaca
