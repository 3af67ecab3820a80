/*
 * Oracle: Galerkin P0 single layer entries V_ij(s) = int_{tau_i} int_{tau_j} G_s(|x - y|)
 * dS_y dS_x (paper Sec. 3, eq. bie_semi_indirect, Laplace-domain kernel of Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY -- plain FP64 loops; shares no code with the GPU library.
 *
 * Quadrature reading (the paper treats the weakly singular Galerkin integrals with the
 * regularising transformations of Erichsen and Sauter and the regular ones with a
 * distance heuristic, without orders):
 *   far blocks, and disjoint near pairs with q >= 4:  6-point rule x 6-point rule;
 *   disjoint near pairs with 2 <= q < 4:              collapsed 4x4 x collapsed 4x4;
 *   disjoint near pairs with q < 2 (no shared vertex): outer collapsed n_G x n_G rule on
 *       tau_i, inner integral over tau_j split at the point of tau_j nearest to the outer
 *       point into three Duffy sub-triangles with n_G x n_G points each;
 *   pairs sharing an edge or a vertex: the Sauter-Schwab regularising maps of [0,1]^4
 *       (the family of the Erichsen-Sauter scheme).  Both triangles are mapped from the
 *       reference triangle {0 <= t2 <= t1 <= 1} by x(t) = P0 + t1 (P1 - P0) + t2 (P2 - P1)
 *       with the shared vertex at P0 (and, for an edge, the shared edge at t2 = 0).  The
 *       product of the two reference triangles splits into 2 (vertex) or 5 (edge) regions,
 *       each mapped from (xi, eta1, eta2, eta3) in [0,1]^4 so that x - y = xi d(eta)
 *       (vertex) or xi eta1 d(eta2, eta3) (edge) with |d| bounded away from zero.  The
 *       kernel depends on xi (and eta1) only through exp(-s r) / r, so these integrals are
 *       done exactly: vertex int_0^1 xi^2 e^{-t xi} d xi = phi2(t) =
 *       (2 - e^{-t}(t^2 + 2t + 2)) / t^3 (series sum_k (-t)^k / (k! (k + 3)) for |t| <= 1),
 *       edge int_0^1 eta1 phi2(t eta1) d eta1 = (t - 2 + e^{-t}(t + 2)) / t^3 (series
 *       sum_k (-t)^k / (k! (k + 2) (k + 3)) for |t| <= 1); the remaining smooth integral
 *       over (eta1, eta2, eta3) (vertex) or (eta2, eta3) (edge) takes n_S Gauss-Legendre
 *       points per direction;
 *   coincident pairs (i == j): exact reduction to one angle.  For a flat triangle T the
 *       kernel depends on z = x - y only, so V = int k(z) |T cap (T + z)| dz, and with the
 *       barycentric functions l_i (linear parts ell_i) |T cap (T + z)| =
 *       A (1 - sum_i max(0, ell_i(z)))^2.  In polar coordinates z = rho e_theta this is
 *       V = A/(4 pi) int_0^{2 pi} R(theta) psi(s R(theta)) dtheta with
 *       R = 1 / sum_i max(0, ell_i(e_theta)) and psi(t) = int_0^1 e^{-t u} (1 - u)^2 du
 *       = 1/t - 2/t^2 + 2/t^3 - 2 e^{-t}/t^3 (series 2 sum_k (-t)^k / (k + 3)! for small t);
 *       the six sectors between the edge directions are integrated with n_theta
 *       Gauss-Legendre points each.
 *   q = |x_i - x_j| / max(h_i, h_j).
 * Vertex order of the touching maps: for a shared edge, P0 and P1 are the shared vertices
 * in the order they appear in tau_i's vertex list and P2 each triangle's third vertex;
 * for a shared vertex V, each triangle's list is rotated cyclically to start at V.
 *
 * Parity pins: tests/test_oracle_galerkin.py.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define PI 3.14159265358979323846

typedef struct {
    double v[3][3];   /* vertices */
    double x[3];      /* centroid */
    double area, h;
} gtri_t;

static void sub3(const double *p, const double *q, double *r) {
    r[0] = p[0] - q[0]; r[1] = p[1] - q[1]; r[2] = p[2] - q[2];
}
static double dot3(const double *p, const double *q) {
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
}
static void cross3(const double *p, const double *q, double *r) {
    r[0] = p[1] * q[2] - p[2] * q[1];
    r[1] = p[2] * q[0] - p[0] * q[2];
    r[2] = p[0] * q[1] - p[1] * q[0];
}
static double norm3(const double *p) { return sqrt(dot3(p, p)); }

static void make_gtri(const double *v9, gtri_t *t) {
    double e1[3], e2[3], e3[3], nn[3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) t->v[a][k] = v9[3 * a + k];
    for (int k = 0; k < 3; ++k) t->x[k] = (t->v[0][k] + t->v[1][k] + t->v[2][k]) / 3.0;
    sub3(t->v[1], t->v[0], e1);
    sub3(t->v[2], t->v[0], e2);
    sub3(t->v[2], t->v[1], e3);
    cross3(e1, e2, nn);
    t->area = 0.5 * norm3(nn);
    double h = norm3(e1), h2 = norm3(e2), h3 = norm3(e3);
    if (h2 > h) h = h2;
    if (h3 > h) h = h3;
    t->h = h;
}

typedef struct {
    int n;
    double *y, *w;
} pts_t;

static void push(pts_t *q, const double *y, double w) {
    q->y[3 * q->n] = y[0];
    q->y[3 * q->n + 1] = y[1];
    q->y[3 * q->n + 2] = y[2];
    q->w[q->n] = w;
    q->n++;
}

static void rule6(const gtri_t *t, const double *r6, pts_t *q) {
    for (int p = 0; p < 6; ++p) {
        double y[3];
        for (int k = 0; k < 3; ++k)
            y[k] = r6[4 * p] * t->v[0][k] + r6[4 * p + 1] * t->v[1][k] + r6[4 * p + 2] * t->v[2][k];
        push(q, y, r6[4 * p + 3] * t->area);
    }
}

/* collapsed n x n rule on (a, b, c) collapsed at a */
static void collapsed(const double *a, const double *b, const double *c, int n, const double *g,
                      pts_t *q) {
    double e1[3], e2[3], nn[3];
    sub3(b, a, e1);
    sub3(c, b, e2);
    cross3(e1, e2, nn);
    double two_area = norm3(nn);
    for (int iu = 0; iu < n; ++iu)
        for (int iv = 0; iv < n; ++iv) {
            double u = g[2 * iu], v = g[2 * iv];
            double y[3];
            for (int k = 0; k < 3; ++k) y[k] = a[k] + u * e1[k] + u * v * e2[k];
            push(q, y, g[2 * iu + 1] * g[2 * iv + 1] * u * two_area);
        }
}

/* closest point of triangle (a, b, c) to x (Voronoi-region test on the barycentric form) */
static void closest_point(const double *x, const double *a, const double *b, const double *c,
                          double *p) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    sub3(x, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { for (int k = 0; k < 3; ++k) p[k] = a[k]; return; }
    sub3(x, b, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { for (int k = 0; k < 3; ++k) p[k] = b[k]; return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + v * ab[k];
        return;
    }
    sub3(x, c, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { for (int k = 0; k < 3; ++k) p[k] = c[k]; return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + w * ac[k];
        return;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int k = 0; k < 3; ++k) p[k] = b[k] + w * (c[k] - b[k]);
        return;
    }
    double denom = 1.0 / (va + vb + vc);
    double v = vb * denom, w = vc * denom;
    for (int k = 0; k < 3; ++k) p[k] = a[k] + ab[k] * v + ac[k] * w;
}

static void accumulate(const double *x, double wx, const pts_t *inner, int L,
                       const double *s_re, const double *s_im, double *acc) {
    for (int p = 0; p < inner->n; ++p) {
        double dv[3];
        sub3(x, inner->y + 3 * p, dv);
        double r = norm3(dv);
        double w = wx * inner->w[p] / (4.0 * PI * r);
        for (int l = 0; l < L; ++l) {
            double mag = exp(-s_re[l] * r);
            acc[2 * l] += w * mag * cos(s_im[l] * r);
            acc[2 * l + 1] -= w * mag * sin(s_im[l] * r);
        }
    }
}

/* psi(t) = int_0^1 e^{-t u} (1 - u)^2 du */
static double complex psi(double complex t) {
    if (cabs(t) < 2.0) {
        double complex term = 1.0, sum = 0.0;
        double fact = 6.0;   /* (k + 3)! */
        for (int k = 0; k < 40; ++k) {
            sum += 2.0 * term / fact;
            term *= -t;
            fact *= (double)(k + 4);
        }
        return sum;
    }
    return 1.0 / t - 2.0 / (t * t) + 2.0 / (t * t * t) - 2.0 * cexp(-t) / (t * t * t);
}

/* Coincident entry by the angular reduction (n_theta Gauss points per sector). */
static void coincident(const gtri_t *t, int L, const double *s_re, const double *s_im, int nt,
                       const double *gt, double *out) {
    /* in-plane frame */
    double e1[3], e2[3], nn[3], f1[3], f2[3];
    sub3(t->v[1], t->v[0], e1);
    sub3(t->v[2], t->v[0], e2);
    cross3(e1, e2, nn);
    double ln = norm3(e1);
    for (int k = 0; k < 3; ++k) f1[k] = e1[k] / ln;
    double nl = norm3(nn);
    double un[3] = {nn[0] / nl, nn[1] / nl, nn[2] / nl};
    cross3(un, f1, f2);
    /* 2-D vertices */
    double P[3][2];
    for (int a = 0; a < 3; ++a) {
        double d[3];
        sub3(t->v[a], t->v[0], d);
        P[a][0] = dot3(d, f1);
        P[a][1] = dot3(d, f2);
    }
    /* gradients of the barycentric functions: grad l_a = rot90(P_c - P_b) / (2 A) oriented */
    double A2 = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]);
    double G[3][2];
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        G[a][0] = (P[b][1] - P[c][1]) / A2;
        G[a][1] = (P[c][0] - P[b][0]) / A2;
    }
    /* breakpoints: directions where some ell_a(e_theta) = G_a . e_theta changes sign */
    double th[6];
    int nb = 0;
    for (int a = 0; a < 3; ++a) {
        double base = atan2(G[a][1], G[a][0]);
        double t1 = base + 0.5 * PI, t2 = base - 0.5 * PI;
        th[nb++] = fmod(t1 + 4.0 * PI, 2.0 * PI);
        th[nb++] = fmod(t2 + 4.0 * PI, 2.0 * PI);
    }
    /* sort */
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            if (th[j] < th[i]) { double tmp = th[i]; th[i] = th[j]; th[j] = tmp; }
    for (int l = 0; l < L; ++l) {
        double complex s = s_re[l] + I * s_im[l];
        double complex acc = 0.0;
        for (int sec = 0; sec < 6; ++sec) {
            double ta = th[sec], tb = (sec == 5) ? th[0] + 2.0 * PI : th[sec + 1];
            if (tb - ta <= 0.0) continue;
            for (int q = 0; q < nt; ++q) {
                double theta = ta + (tb - ta) * gt[2 * q];
                double w = (tb - ta) * gt[2 * q + 1];
                double c = cos(theta), sn = sin(theta);
                double g = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double e = G[a][0] * c + G[a][1] * sn;
                    if (e > 0.0) g += e;
                }
                double R = 1.0 / g;
                acc += w * R * psi(s * R);
            }
        }
        acc *= t->area / (4.0 * PI);
        out[2 * l] = creal(acc);
        out[2 * l + 1] = cimag(acc);
    }
}


/* phi2(t) = int_0^1 xi^2 e^{-t xi} d xi */
static double complex phi2(double complex t) {
    if (cabs(t) <= 1.0) {
        double complex term = 1.0, sum = 0.0;   /* term = (-t)^k / k! */
        for (int k = 0; k < 30; ++k) {
            sum += term / (double)(k + 3);
            term *= -t / (double)(k + 1);
        }
        return sum;
    }
    return (2.0 - cexp(-t) * (t * t + 2.0 * t + 2.0)) / (t * t * t);
}

/* one region term of the vertex maps: weight * phi2(s rho) / (4 pi rho), every frequency */
static void ss_add(const double *d, double wg, int L, const double *s_re, const double *s_im,
                   double *acc) {
    double rho = norm3(d);
    for (int l = 0; l < L; ++l) {
        double complex s = s_re[l] + I * s_im[l];
        double complex v = wg * phi2(s * rho) / (4.0 * PI * rho);
        acc[2 * l] += creal(v);
        acc[2 * l + 1] += cimag(v);
    }
}

/* Common vertex V: tau_i = (V, a1, a2), tau_j = (V, b1, b2). */
static void ss_vertex(const double *V, const double *a1, const double *a2, const double *b1,
                      const double *b2, double area_i, double area_j, int n, const double *g,
                      int L, const double *s_re, const double *s_im, double *out) {
    double X1[3], X2[3], Y1[3], Y2[3];
    sub3(a1, V, X1);
    sub3(a2, a1, X2);
    sub3(b1, V, Y1);
    sub3(b2, b1, Y2);
    for (int l = 0; l < 2 * L; ++l) out[l] = 0.0;
    for (int p1 = 0; p1 < n; ++p1)
        for (int p2 = 0; p2 < n; ++p2)
            for (int p3 = 0; p3 < n; ++p3) {
                double e1 = g[2 * p1], e2 = g[2 * p2], e3 = g[2 * p3];
                double w = g[2 * p1 + 1] * g[2 * p2 + 1] * g[2 * p3 + 1];
                double d[3];
                /* region t1 >= u1: t = xi (1, e1), u = xi e2 (1, e3) */
                for (int k = 0; k < 3; ++k)
                    d[k] = (X1[k] + e1 * X2[k]) - e2 * (Y1[k] + e3 * Y2[k]);
                ss_add(d, w * e2, L, s_re, s_im, out);
                /* region u1 > t1: u = xi (1, e1), t = xi e2 (1, e3) */
                for (int k = 0; k < 3; ++k)
                    d[k] = e2 * (X1[k] + e3 * X2[k]) - (Y1[k] + e1 * Y2[k]);
                ss_add(d, w * e2, L, s_re, s_im, out);
            }
    for (int l = 0; l < 2 * L; ++l) out[l] *= 4.0 * area_i * area_j;
}

/* Phi(t) = int_0^1 eta int_0^1 xi^2 e^{-t eta xi} d xi d eta = (t - 2 + e^{-t} (t + 2)) / t^3 */
static double complex phi_edge(double complex t) {
    if (cabs(t) <= 1.0) {
        double complex term = 1.0, sum = 0.0;   /* term = (-t)^k / k! */
        for (int k = 0; k < 30; ++k) {
            sum += term / ((double)(k + 2) * (double)(k + 3));
            term *= -t / (double)(k + 1);
        }
        return sum;
    }
    return (t - 2.0 + cexp(-t) * (t + 2.0)) / (t * t * t);
}

/* Common edge (P0, P1): tau_i = (P0, P1, a), tau_j = (P0, P1, b).  In every region
 * x - y = xi eta1 d(eta2, eta3), so both the xi and the eta1 integral are exact (phi_edge)
 * and n x n Gauss points remain per region. */
static void ss_edge(const double *P0, const double *P1, const double *a, const double *b,
                    double area_i, double area_j, int n, const double *g, int L,
                    const double *s_re, const double *s_im, double *out) {
    double E[3], A[3], B[3];
    sub3(P1, P0, E);
    sub3(a, P1, A);
    sub3(b, P1, B);
    for (int l = 0; l < 2 * L; ++l) out[l] = 0.0;
    for (int p2 = 0; p2 < n; ++p2)
        for (int p3 = 0; p3 < n; ++p3) {
            double e2 = g[2 * p2], e3 = g[2 * p3];
            double w = g[2 * p2 + 1] * g[2 * p3 + 1];
            double c[5][3] = {{e2, e3, -(1.0 - e2)},
                              {e2 * e3, 1.0, -e2 * (1.0 - e3)},
                              {-e2, 1.0 - e2, -e2 * e3},
                              {-e2 * e3, e2 * (1.0 - e3), -1.0},
                              {-e2 * e3, 1.0 - e2 * e3, -e2}};
            for (int r = 0; r < 5; ++r) {
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = c[r][0] * E[k] + c[r][1] * A[k] + c[r][2] * B[k];
                double rho = norm3(d), wr = w * (r == 0 ? 1.0 : e2);
                for (int l = 0; l < L; ++l) {
                    double complex s = s_re[l] + I * s_im[l];
                    double complex v = wr * phi_edge(s * rho) / (4.0 * PI * rho);
                    out[2 * l] += creal(v);
                    out[2 * l + 1] += cimag(v);
                }
            }
        }
    for (int l = 0; l < 2 * L; ++l) out[l] *= 4.0 * area_i * area_j;
}

enum { G_FAR36 = 0, G_MID = 1, G_NEAR = 2, G_EDGE = 3, G_VERTEX = 4, G_COINC = 5 };

/*
 * tri9: M x 9 vertex coordinates; tri: M x 3 vertex ids (for the shared-vertex test);
 * far[p] = 1 for pairs of admissible blocks; out: npair x L x 2.
 */
void oracle_galerkin_entries(const double *tri9, const int32_t *tri, int L, const double *s_re,
                             const double *s_im, int64_t npair, const int64_t *ii,
                             const int64_t *jj, const int32_t *far, const double *r6,
                             int n4, const double *g4, int ng, const double *gg, int nt,
                             const double *gt, int nss, const double *gs, double *out,
                             int32_t *tier_out) {
    int maxq = 3 * ng * ng;
    if (n4 * n4 > maxq) maxq = n4 * n4;
    if (maxq < 6) maxq = 6;
    int maxo = ng * ng;
    if (n4 * n4 > maxo) maxo = n4 * n4;
    if (maxo < 6) maxo = 6;
#pragma omp parallel
    {
        pts_t qin, qout;
        qin.y = (double *)malloc(sizeof(double) * 3 * maxq);
        qin.w = (double *)malloc(sizeof(double) * maxq);
        qout.y = (double *)malloc(sizeof(double) * 3 * maxo);
        qout.w = (double *)malloc(sizeof(double) * maxo);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npair; ++p) {
            gtri_t ti, tj;
            const int64_t i = ii[p], j = jj[p];
            make_gtri(tri9 + 9 * i, &ti);
            make_gtri(tri9 + 9 * j, &tj);
            double *o = out + 2 * (size_t)L * p;
            for (int l = 0; l < 2 * L; ++l) o[l] = 0.0;
            /* shared vertices: positions in tau_i (ascending) and in tau_j */
            int shared = 0, pos_i[3], pos_j[3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    if (tri[3 * i + a] == tri[3 * j + b]) {
                        pos_i[shared] = a;
                        pos_j[shared] = b;
                        ++shared;
                    }
            int tier;
            if (i == j) tier = G_COINC;
            else if (far[p]) tier = G_FAR36;
            else if (shared == 2) tier = G_EDGE;
            else if (shared == 1) tier = G_VERTEX;
            else {
                double dv[3];
                sub3(ti.x, tj.x, dv);
                double hm = ti.h > tj.h ? ti.h : tj.h;
                double q = norm3(dv) / hm;
                tier = q >= 4.0 ? G_FAR36 : (q >= 2.0 ? G_MID : G_NEAR);
            }
            if (tier_out) tier_out[p] = tier;
            if (tier == G_COINC) {
                coincident(&tj, L, s_re, s_im, nt, gt, o);
                continue;
            }
            qout.n = 0;
            if (tier == G_FAR36 || tier == G_MID) {
                qin.n = 0;
                if (tier == G_FAR36) {
                    rule6(&ti, r6, &qout);
                    rule6(&tj, r6, &qin);
                } else {
                    collapsed(ti.v[0], ti.v[1], ti.v[2], n4, g4, &qout);
                    collapsed(tj.v[0], tj.v[1], tj.v[2], n4, g4, &qin);
                }
                for (int a = 0; a < qout.n; ++a) accumulate(qout.y + 3 * a, qout.w[a], &qin, L, s_re, s_im, o);
                continue;
            }
            if (tier == G_EDGE) {
                int ta = 3 - pos_i[0] - pos_i[1], tb = 3 - pos_j[0] - pos_j[1];
                ss_edge(ti.v[pos_i[0]], ti.v[pos_i[1]], ti.v[ta], tj.v[tb], ti.area, tj.area, nss,
                        gs, L, s_re, s_im, o);
                continue;
            }
            if (tier == G_VERTEX) {
                int a = pos_i[0], b = pos_j[0];
                ss_vertex(ti.v[a], ti.v[(a + 1) % 3], ti.v[(a + 2) % 3], tj.v[(b + 1) % 3],
                          tj.v[(b + 2) % 3], ti.area, tj.area, nss, gs, L, s_re, s_im, o);
                continue;
            }
            /* disjoint q < 2: outer collapsed rule at vertex a of tau_i, inner split at the
             * nearest point */
            collapsed(ti.v[0], ti.v[1], ti.v[2], ng, gg, &qout);
            for (int a = 0; a < qout.n; ++a) {
                const double *x = qout.y + 3 * a;
                double pnt[3];
                closest_point(x, tj.v[0], tj.v[1], tj.v[2], pnt);
                qin.n = 0;
                collapsed(pnt, tj.v[1], tj.v[2], ng, gg, &qin);
                collapsed(pnt, tj.v[2], tj.v[0], ng, gg, &qin);
                collapsed(pnt, tj.v[0], tj.v[1], ng, gg, &qin);
                accumulate(x, qout.w[a], &qin, L, s_re, s_im, o);
            }
        }
        free(qin.y);
        free(qin.w);
        free(qout.y);
        free(qout.w);
    }
}
