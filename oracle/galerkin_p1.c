/*
 * Oracle: Galerkin operators of the Neumann problem with linear continuous test and trial
 * functions (paper Sec. 3, eq. bie_semi_neum), Laplace-domain kernel G_s = e^{-s r}/(4 pi r):
 *
 *   adjoint double layer  K'_ij(s) = int int phi_i(x) dG/dn_x(x - y) phi_j(y) dS_y dS_x,
 *       dG/dn_x = -((x - y) . n_x) e^{-s r} (1 + s r) / (4 pi r^3);
 *   hypersingular         D_ij(s)  = int int G_s(x - y) [curl phi_i(x) . curl phi_j(y)
 *                                        + s^2 (n_x . n_y) phi_i(x) phi_j(y)] dS_y dS_x,
 *       the hypersingular form after integration by parts (the Laplace-domain counterpart of
 *       Maue's formula for the Helmholtz operator, wave number k = i s): the finite-part
 *       integral of the paper's definition reduces to weakly singular integrals of G_s.
 *
 * TEST INFRASTRUCTURE ONLY -- plain FP64 loops; shares no code with the GPU library.
 *
 * Entries are sums over the triangle pairs (tau, tau') of the supports of phi_i and phi_j of
 * the local integrals M_ab = int_tau int_tau' k(x, y) lambda_a(x) lambda_b(y), lambda the
 * barycentric coordinates (phi restricted to a triangle), and for D the constant surface
 * curls curl lambda_a = -e_a / (2 A) (e_a the edge opposite to vertex a, oriented
 * counter-clockwise seen from outside).
 *
 * Quadrature per triangle pair (the paper's reading for the Galerkin single layer, extended
 * to the weights lambda_a lambda_b):
 *   far blocks and disjoint pairs with q >= 4: 6-point x 6-point rule;
 *   disjoint pairs with 2 <= q < 4: collapsed 4 x 4 x collapsed 4 x 4;
 *   disjoint pairs with q < 2: outer collapsed n_G x n_G on tau, inner integral over tau'
 *       split at the point of tau' nearest to the outer point into three Duffy triangles;
 *   identical triangles, a shared edge, a shared vertex: the regularising maps of Sauter
 *       and Schwab from [0,1]^4 (6, 5 and 2 regions), every variable with n_S Gauss points
 *       (numerically: the weights lambda_a lambda_b make the radial integrals polynomial
 *       times e^{-s r} / r, so no closed form is used here).
 *   q = |c_tau - c_tau'| / max(h, h').  Both triangles are mapped from the reference triangle
 *   {0 <= t2 <= t1 <= 1} by x(t) = P0 + t1 (P1 - P0) + t2 (P2 - P1), lambda = (1 - t1,
 *   t1 - t2, t2) for (P0, P1, P2); identical: the triangle's own order; shared edge: P0, P1
 *   the shared vertices in tau's order, P2 the third vertex of each; shared vertex: each
 *   list rotated to start there.  The dG/dn_x integrand of a coplanar pair is 0.
 *
 * Parity pins: tests/test_oracle_galerkin_p1.py.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

typedef struct {
    double v[3][3];
    double n[3], c[3];
    double area, h;
} ptri_t;

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

static void make_ptri(const double *xyz, const int32_t *tv, ptri_t *t) {
    double e1[3], e2[3], e3[3], nn[3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) t->v[a][k] = xyz[3 * (int64_t)tv[a] + k];
    for (int k = 0; k < 3; ++k) t->c[k] = (t->v[0][k] + t->v[1][k] + t->v[2][k]) / 3.0;
    sub3(t->v[1], t->v[0], e1);
    sub3(t->v[2], t->v[0], e2);
    sub3(t->v[2], t->v[1], e3);
    cross3(e1, e2, nn);
    double len = norm3(nn);
    t->area = 0.5 * len;
    for (int k = 0; k < 3; ++k) t->n[k] = nn[k] / len;
    double h = norm3(e1), h2 = norm3(e2), h3 = norm3(e3);
    if (h2 > h) h = h2;
    if (h3 > h) h = h3;
    t->h = h;
}

/* barycentric coordinates of y (a point of t's plane) */
static void bary(const ptri_t *t, const double *y, double *lam) {
    double e1[3], e2[3], d[3];
    sub3(t->v[1], t->v[0], e1);
    sub3(t->v[2], t->v[0], e2);
    sub3(y, t->v[0], d);
    double a = dot3(e1, e1), b = dot3(e1, e2), c = dot3(e2, e2);
    double p = dot3(d, e1), q = dot3(d, e2);
    double det = a * c - b * b;
    double u = (c * p - b * q) / det, v = (a * q - b * p) / det;
    lam[0] = 1.0 - u - v;
    lam[1] = u;
    lam[2] = v;
}

/* point list on one triangle: positions, weights (with the surface measure), lambda */
typedef struct {
    int n;
    double *y, *w, *lam;
} plist_t;

static void ppush(plist_t *q, const double *y, double w, const double *lam) {
    memcpy(q->y + 3 * q->n, y, 3 * sizeof(double));
    memcpy(q->lam + 3 * q->n, lam, 3 * sizeof(double));
    q->w[q->n] = w;
    q->n++;
}

static void rule6_p(const ptri_t *t, const double *r6, plist_t *q) {
    for (int p = 0; p < 6; ++p) {
        double y[3], lam[3] = {r6[4 * p], r6[4 * p + 1], r6[4 * p + 2]};
        for (int k = 0; k < 3; ++k)
            y[k] = lam[0] * t->v[0][k] + lam[1] * t->v[1][k] + lam[2] * t->v[2][k];
        ppush(q, y, r6[4 * p + 3] * t->area, lam);
    }
}

/* collapsed n x n rule on the sub-triangle (a, b, c) of t (collapsed at a) */
static void collapsed_p(const ptri_t *t, const double *a, const double *b, const double *c,
                        int n, const double *g, plist_t *q) {
    double e1[3], e2[3], nn[3];
    sub3(b, a, e1);
    sub3(c, b, e2);
    cross3(e1, e2, nn);
    double two_area = norm3(nn);
    for (int iu = 0; iu < n; ++iu)
        for (int iv = 0; iv < n; ++iv) {
            double u = g[2 * iu], v = g[2 * iv], y[3], lam[3];
            for (int k = 0; k < 3; ++k) y[k] = a[k] + u * e1[k] + u * v * e2[k];
            bary(t, y, lam);
            ppush(q, y, g[2 * iu + 1] * g[2 * iv + 1] * u * two_area, lam);
        }
}

/* closest point of triangle (a, b, c) to x */
static void closest_pt(const double *x, const double *a, const double *b, const double *c,
                       double *p) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    sub3(x, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { memcpy(p, a, 3 * sizeof(double)); return; }
    sub3(x, b, bp);
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { memcpy(p, b, 3 * sizeof(double)); return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + v * ab[k];
        return;
    }
    sub3(x, c, cp);
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { memcpy(p, c, 3 * sizeof(double)); return; }
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

/* kernel value at every frequency: kind 0 G_s, kind 1 dG/dn_x */
static void kernel_l(int kind, const double *x, const double *y, const double *nx, int L,
                     const double *s_re, const double *s_im, double complex *out) {
    double d[3];
    sub3(x, y, d);
    double r = norm3(d);
    double num = kind == 1 ? -dot3(d, nx) : 0.0;
    for (int l = 0; l < L; ++l) {
        double complex s = s_re[l] + I * s_im[l];
        double complex e = cexp(-s * r);
        out[l] = kind == 0 ? e / (4.0 * PI * r) : num * e * (1.0 + s * r) / (4.0 * PI * r * r * r);
    }
}

/* M[(a * 3 + b) * L + l] += w k_l(x, y) lam_x[a] lam_y[b] */
static void add_pt(int kind, const double *x, const double *lx, const double *y, const double *ly,
                   double w, const double *nx, int L, const double *s_re, const double *s_im,
                   double complex *kv, double complex *M) {
    kernel_l(kind, x, y, nx, L, s_re, s_im, kv);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double ww = w * lx[a] * ly[b];
            if (ww == 0.0) continue;
            for (int l = 0; l < L; ++l) M[(a * 3 + b) * L + l] += ww * kv[l];
        }
}

/* reference point t = (t1, t2) of the triangle (P0, P1, P2) -> physical point, lambda */
static void ref_map(const double *P0, const double *P1, const double *P2, double t1, double t2,
                    double *x, double *lam) {
    for (int k = 0; k < 3; ++k) x[k] = P0[k] + t1 * (P1[k] - P0[k]) + t2 * (P2[k] - P1[k]);
    lam[0] = 1.0 - t1;
    lam[1] = t1 - t2;
    lam[2] = t2;
}

/*
 * Touching pair by the regularising maps.  rel: 3 identical, 2 shared edge, 1 shared vertex;
 * (P0, P1, P2) and (Q0, Q1, Q2) the reordered vertices, pa / pb the original local index of
 * each reordered vertex (so lambda of the original vertex pa[c] is the reordered lambda c).
 */
static void touching(int kind, int rel, const double *P[3], const int *pa, const double *Q[3],
                     const int *pb, double ji, double jj, const double *nx, int L,
                     const double *s_re, const double *s_im, int n, const double *g,
                     double complex *kv, double complex *M) {
    for (int i1 = 0; i1 < n; ++i1)
        for (int i2 = 0; i2 < n; ++i2)
            for (int i3 = 0; i3 < n; ++i3)
                for (int i4 = 0; i4 < n; ++i4) {
                    const double xi = g[2 * i1], e1 = g[2 * i2], e2 = g[2 * i3], e3 = g[2 * i4];
                    const double w0 = g[2 * i1 + 1] * g[2 * i2 + 1] * g[2 * i3 + 1] * g[2 * i4 + 1] * ji * jj;
                    double X[6][2], Y[6][2], W[6];
                    int nr = 0;
                    if (rel == 3) {
                        const double jac = xi * xi * xi * e1 * e1 * e2;
                        double A1 = xi, A2 = xi * (1.0 - e1 + e1 * e2);
                        double B1 = xi * (1.0 - e1 * e2 * e3), B2 = xi * (1.0 - e1);
                        X[0][0] = A1; X[0][1] = A2; Y[0][0] = B1; Y[0][1] = B2;
                        X[1][0] = B1; X[1][1] = B2; Y[1][0] = A1; Y[1][1] = A2;
                        double C1 = xi, C2 = xi * e1 * (1.0 - e2 + e2 * e3);
                        double D1 = xi * (1.0 - e1 * e2), D2 = xi * e1 * (1.0 - e2);
                        X[2][0] = C1; X[2][1] = C2; Y[2][0] = D1; Y[2][1] = D2;
                        X[3][0] = D1; X[3][1] = D2; Y[3][0] = C1; Y[3][1] = C2;
                        double E1 = xi * (1.0 - e1 * e2 * e3), E2 = xi * e1 * (1.0 - e2 * e3);
                        double F1 = xi, F2 = xi * e1 * (1.0 - e2);
                        X[4][0] = E1; X[4][1] = E2; Y[4][0] = F1; Y[4][1] = F2;
                        X[5][0] = F1; X[5][1] = F2; Y[5][0] = E1; Y[5][1] = E2;
                        for (int r = 0; r < 6; ++r) W[r] = jac;
                        nr = 6;
                    } else if (rel == 2) {
                        const double jac = xi * xi * xi * e1 * e1;
                        X[0][0] = xi; X[0][1] = xi * e1 * e3;
                        Y[0][0] = xi * (1.0 - e1 * e2); Y[0][1] = xi * e1 * (1.0 - e2);
                        W[0] = jac;
                        X[1][0] = xi; X[1][1] = xi * e1;
                        Y[1][0] = xi * (1.0 - e1 * e2 * e3); Y[1][1] = xi * e1 * e2 * (1.0 - e3);
                        X[2][0] = xi * (1.0 - e1 * e2); X[2][1] = xi * e1 * (1.0 - e2);
                        Y[2][0] = xi; Y[2][1] = xi * e1 * e2 * e3;
                        X[3][0] = xi * (1.0 - e1 * e2 * e3); X[3][1] = xi * e1 * e2 * (1.0 - e3);
                        Y[3][0] = xi; Y[3][1] = xi * e1;
                        X[4][0] = xi * (1.0 - e1 * e2 * e3); X[4][1] = xi * e1 * (1.0 - e2 * e3);
                        Y[4][0] = xi; Y[4][1] = xi * e1 * e2;
                        for (int r = 1; r < 5; ++r) W[r] = jac * e2;
                        nr = 5;
                    } else {
                        const double jac = xi * xi * xi * e2;
                        X[0][0] = xi; X[0][1] = xi * e1;
                        Y[0][0] = xi * e2; Y[0][1] = xi * e2 * e3;
                        X[1][0] = xi * e2; X[1][1] = xi * e2 * e1;
                        Y[1][0] = xi; Y[1][1] = xi * e3;
                        W[0] = W[1] = jac;
                        nr = 2;
                    }
                    for (int r = 0; r < nr; ++r) {
                        double x[3], y[3], lx[3], ly[3], lxo[3], lyo[3];
                        ref_map(P[0], P[1], P[2], X[r][0], X[r][1], x, lx);
                        ref_map(Q[0], Q[1], Q[2], Y[r][0], Y[r][1], y, ly);
                        for (int c = 0; c < 3; ++c) {
                            lxo[pa[c]] = lx[c];
                            lyo[pb[c]] = ly[c];
                        }
                        add_pt(kind, x, lxo, y, lyo, w0 * W[r], nx, L, s_re, s_im, kv, M);
                    }
                }
}

typedef struct {
    const double *r6;
    int n4; const double *g4;
    int ng; const double *gg;
    int ns; const double *gs;
} prules_t;

/* local matrices M[(a 3 + b) L + l] of the pair (ti, tj) (vertex ids vi, vj) */
static void pair_local(int kind, const double *xyz, const int32_t *vi, const int32_t *vj,
                       int far, const prules_t *R, int L, const double *s_re,
                       const double *s_im, double complex *kv, plist_t *qa, plist_t *qb,
                       plist_t *qc, double complex *M) {
    ptri_t ti, tj;
    make_ptri(xyz, vi, &ti);
    make_ptri(xyz, vj, &tj);
    memset(M, 0, sizeof(double complex) * 9 * L);
    if (kind == 1) {   /* coplanar pair: (x - y) . n_x = 0 on tau_j */
        int cop = 1;
        for (int c = 0; c < 3; ++c) {
            double d[3];
            sub3(tj.v[c], ti.v[0], d);
            if (fabs(dot3(d, ti.n)) > 1e-14 * ti.h) cop = 0;
        }
        if (cop) return;
    }
    int shared = 0, si[3], sj[3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (vi[a] == vj[b]) {
                si[shared] = a;
                sj[shared] = b;
                ++shared;
            }
    if (shared > 0) {
        const double *P[3], *Q[3];
        int pa[3], pb[3];
        if (shared == 3) {
            for (int c = 0; c < 3; ++c) {
                P[c] = ti.v[c]; pa[c] = c;
                Q[c] = ti.v[c]; pb[c] = c;
            }
        } else if (shared == 2) {
            /* shared vertices in tau_i's order */
            int a0 = si[0] < si[1] ? 0 : 1, a1 = 1 - a0;
            pa[0] = si[a0]; pa[1] = si[a1]; pa[2] = 3 - si[0] - si[1];
            pb[0] = sj[a0]; pb[1] = sj[a1]; pb[2] = 3 - sj[0] - sj[1];
            for (int c = 0; c < 3; ++c) { P[c] = ti.v[pa[c]]; Q[c] = tj.v[pb[c]]; }
        } else {
            for (int c = 0; c < 3; ++c) {
                pa[c] = (si[0] + c) % 3;
                pb[c] = (sj[0] + c) % 3;
                P[c] = ti.v[pa[c]];
                Q[c] = tj.v[pb[c]];
            }
        }
        touching(kind, shared, P, pa, Q, pb, 2.0 * ti.area, 2.0 * tj.area, ti.n, L, s_re, s_im,
                 R->ns, R->gs, kv, M);
        return;
    }
    double dv[3];
    sub3(ti.c, tj.c, dv);
    double q = norm3(dv) / (ti.h > tj.h ? ti.h : tj.h);
    qa->n = qb->n = 0;
    if (far || q >= 4.0) {
        rule6_p(&ti, R->r6, qa);
        rule6_p(&tj, R->r6, qb);
    } else if (q >= 2.0) {
        collapsed_p(&ti, ti.v[0], ti.v[1], ti.v[2], R->n4, R->g4, qa);
        collapsed_p(&tj, tj.v[0], tj.v[1], tj.v[2], R->n4, R->g4, qb);
    } else {
        collapsed_p(&ti, ti.v[0], ti.v[1], ti.v[2], R->ng, R->gg, qa);
        for (int p = 0; p < qa->n; ++p) {
            const double *x = qa->y + 3 * p;
            double cp[3];
            closest_pt(x, tj.v[0], tj.v[1], tj.v[2], cp);
            qc->n = 0;
            collapsed_p(&tj, cp, tj.v[1], tj.v[2], R->ng, R->gg, qc);
            collapsed_p(&tj, cp, tj.v[2], tj.v[0], R->ng, R->gg, qc);
            collapsed_p(&tj, cp, tj.v[0], tj.v[1], R->ng, R->gg, qc);
            for (int r = 0; r < qc->n; ++r)
                add_pt(kind, x, qa->lam + 3 * p, qc->y + 3 * r, qc->lam + 3 * r,
                       qa->w[p] * qc->w[r], ti.n, L, s_re, s_im, kv, M);
        }
        return;
    }
    for (int p = 0; p < qa->n; ++p)
        for (int r = 0; r < qb->n; ++r)
            add_pt(kind, qa->y + 3 * p, qa->lam + 3 * p, qb->y + 3 * r, qb->lam + 3 * r,
                   qa->w[p] * qb->w[r], ti.n, L, s_re, s_im, kv, M);
}

/* curl of lambda_a on t: -e_a / (2 A), e_a = v[a+2] - v[a+1] */
static void curl_lam(const ptri_t *t, int a, double *c) {
    int b = (a + 1) % 3, d = (a + 2) % 3;
    for (int k = 0; k < 3; ++k) c[k] = -(t->v[d][k] - t->v[b][k]) / (2.0 * t->area);
}

static plist_t alloc_list(int n) {
    plist_t q;
    q.n = 0;
    q.y = (double *)malloc(sizeof(double) * 3 * n);
    q.w = (double *)malloc(sizeof(double) * n);
    q.lam = (double *)malloc(sizeof(double) * 3 * n);
    return q;
}
static void free_list(plist_t *q) {
    free(q->y);
    free(q->w);
    free(q->lam);
}

/*
 * Entries of the P1 Galerkin operator kind (0: hypersingular D, 1: adjoint double layer K')
 * for vertex pairs (ii[p], jj[p]) at every frequency: out npair x L x 2.  pptr / ptri / ploc:
 * each vertex's triangles and its local index in them; far[p]: admissible-block pair.
 */
void oracle_p1_galerkin_entries(int op, const double *xyz, const int32_t *tri,
                                const int64_t *pptr, const int32_t *ptri, const int32_t *ploc,
                                int L, const double *s_re, const double *s_im, int64_t npair,
                                const int64_t *ii, const int64_t *jj, const int32_t *far,
                                const double *r6, int n4, const double *g4, int ng,
                                const double *gg, int ns, const double *gs, double *out) {
    prules_t R = {r6, n4, g4, ng, gg, ns, gs};
    int maxq = 6;
    if (n4 * n4 > maxq) maxq = n4 * n4;
    if (3 * ng * ng > maxq) maxq = 3 * ng * ng;
#pragma omp parallel
    {
        plist_t qa = alloc_list(maxq), qb = alloc_list(maxq), qc = alloc_list(maxq);
        double complex *kv = (double complex *)malloc(sizeof(double complex) * L);
        double complex *M = (double complex *)malloc(sizeof(double complex) * 9 * L);
        double complex *acc = (double complex *)malloc(sizeof(double complex) * L);
#pragma omp for schedule(dynamic, 4)
        for (int64_t p = 0; p < npair; ++p) {
            for (int l = 0; l < L; ++l) acc[l] = 0.0;
            for (int64_t e = pptr[ii[p]]; e < pptr[ii[p] + 1]; ++e)
                for (int64_t f = pptr[jj[p]]; f < pptr[jj[p] + 1]; ++f) {
                    const int32_t *vi = tri + 3 * (int64_t)ptri[e], *vj = tri + 3 * (int64_t)ptri[f];
                    const int a = ploc[e], b = ploc[f];
                    pair_local(op == 0 ? 0 : 1, xyz, vi, vj, far[p], &R, L, s_re, s_im, kv, &qa,
                               &qb, &qc, M);
                    if (op == 1) {
                        for (int l = 0; l < L; ++l) acc[l] += M[(a * 3 + b) * L + l];
                    } else {
                        ptri_t ti, tj;
                        make_ptri(xyz, vi, &ti);
                        make_ptri(xyz, vj, &tj);
                        double ca[3], cb[3];
                        curl_lam(&ti, a, ca);
                        curl_lam(&tj, b, cb);
                        const double cc = dot3(ca, cb), nn = dot3(ti.n, tj.n);
                        for (int l = 0; l < L; ++l) {
                            double complex s = s_re[l] + I * s_im[l], S = 0.0;
                            for (int k = 0; k < 9; ++k) S += M[k * L + l];
                            acc[l] += cc * S + s * s * nn * M[(a * 3 + b) * L + l];
                        }
                    }
                }
            for (int l = 0; l < L; ++l) {
                out[2 * ((size_t)p * L + l)] = creal(acc[l]);
                out[2 * ((size_t)p * L + l) + 1] = cimag(acc[l]);
            }
        }
        free_list(&qa);
        free_list(&qb);
        free_list(&qc);
        free(kv);
        free(M);
        free(acc);
    }
}

/*
 * Local matrices of single triangle pairs (test hook): kind 0 G_s, kind 1 dG/dn_x; out
 * npair x 9 x L x 2 (a 3 + b, lambda_a on tri[ti[p]], lambda_b on tri[tj[p]]).
 */
void oracle_p1_pair_local(int kind, const double *xyz, const int32_t *tri, int L,
                          const double *s_re, const double *s_im, int64_t npair,
                          const int64_t *ti, const int64_t *tj, const int32_t *far,
                          const double *r6, int n4, const double *g4, int ng, const double *gg,
                          int ns, const double *gs, double *out) {
    prules_t R = {r6, n4, g4, ng, gg, ns, gs};
    int maxq = 6;
    if (n4 * n4 > maxq) maxq = n4 * n4;
    if (3 * ng * ng > maxq) maxq = 3 * ng * ng;
    plist_t qa = alloc_list(maxq), qb = alloc_list(maxq), qc = alloc_list(maxq);
    double complex *kv = (double complex *)malloc(sizeof(double complex) * L);
    double complex *M = (double complex *)malloc(sizeof(double complex) * 9 * L);
    for (int64_t p = 0; p < npair; ++p) {
        pair_local(kind, xyz, tri + 3 * ti[p], tri + 3 * tj[p], far[p], &R, L, s_re, s_im, kv,
                   &qa, &qb, &qc, M);
        for (int k = 0; k < 9 * L; ++k) {
            out[2 * ((size_t)p * 9 * L + k)] = creal(M[k]);
            out[2 * ((size_t)p * 9 * L + k) + 1] = cimag(M[k]);
        }
    }
    free_list(&qa);
    free_list(&qb);
    free_list(&qc);
    free(kv);
    free(M);
}

/* Sauter-Schwab maps on a smooth integrand f(x_hat, y_hat) = product of monomials (test
 * hook for the maps alone): returns int_T int_T x1^a x2^b y1^c y2^d over the reference
 * triangle pair for the relation rel (3 identical, 2 edge, 1 vertex) with the reference
 * coordinates as they enter the maps. */
double oracle_ss_monomial(int rel, int a, int b, int c, int d, int n, const double *g) {
    double sum = 0.0;
    for (int i1 = 0; i1 < n; ++i1)
        for (int i2 = 0; i2 < n; ++i2)
            for (int i3 = 0; i3 < n; ++i3)
                for (int i4 = 0; i4 < n; ++i4) {
                    const double xi = g[2 * i1], e1 = g[2 * i2], e2 = g[2 * i3], e3 = g[2 * i4];
                    const double w0 = g[2 * i1 + 1] * g[2 * i2 + 1] * g[2 * i3 + 1] * g[2 * i4 + 1];
                    double X[6][2], Y[6][2], W[6];
                    int nr;
                    if (rel == 3) {
                        const double jac = xi * xi * xi * e1 * e1 * e2;
                        double A1 = xi, A2 = xi * (1.0 - e1 + e1 * e2);
                        double B1 = xi * (1.0 - e1 * e2 * e3), B2 = xi * (1.0 - e1);
                        X[0][0] = A1; X[0][1] = A2; Y[0][0] = B1; Y[0][1] = B2;
                        X[1][0] = B1; X[1][1] = B2; Y[1][0] = A1; Y[1][1] = A2;
                        double C1 = xi, C2 = xi * e1 * (1.0 - e2 + e2 * e3);
                        double D1 = xi * (1.0 - e1 * e2), D2 = xi * e1 * (1.0 - e2);
                        X[2][0] = C1; X[2][1] = C2; Y[2][0] = D1; Y[2][1] = D2;
                        X[3][0] = D1; X[3][1] = D2; Y[3][0] = C1; Y[3][1] = C2;
                        double E1 = xi * (1.0 - e1 * e2 * e3), E2 = xi * e1 * (1.0 - e2 * e3);
                        double F1 = xi, F2 = xi * e1 * (1.0 - e2);
                        X[4][0] = E1; X[4][1] = E2; Y[4][0] = F1; Y[4][1] = F2;
                        X[5][0] = F1; X[5][1] = F2; Y[5][0] = E1; Y[5][1] = E2;
                        for (int r = 0; r < 6; ++r) W[r] = jac;
                        nr = 6;
                    } else if (rel == 2) {
                        const double jac = xi * xi * xi * e1 * e1;
                        X[0][0] = xi; X[0][1] = xi * e1 * e3;
                        Y[0][0] = xi * (1.0 - e1 * e2); Y[0][1] = xi * e1 * (1.0 - e2);
                        W[0] = jac;
                        X[1][0] = xi; X[1][1] = xi * e1;
                        Y[1][0] = xi * (1.0 - e1 * e2 * e3); Y[1][1] = xi * e1 * e2 * (1.0 - e3);
                        X[2][0] = xi * (1.0 - e1 * e2); X[2][1] = xi * e1 * (1.0 - e2);
                        Y[2][0] = xi; Y[2][1] = xi * e1 * e2 * e3;
                        X[3][0] = xi * (1.0 - e1 * e2 * e3); X[3][1] = xi * e1 * e2 * (1.0 - e3);
                        Y[3][0] = xi; Y[3][1] = xi * e1;
                        X[4][0] = xi * (1.0 - e1 * e2 * e3); X[4][1] = xi * e1 * (1.0 - e2 * e3);
                        Y[4][0] = xi; Y[4][1] = xi * e1 * e2;
                        for (int r = 1; r < 5; ++r) W[r] = jac * e2;
                        nr = 5;
                    } else {
                        const double jac = xi * xi * xi * e2;
                        X[0][0] = xi; X[0][1] = xi * e1;
                        Y[0][0] = xi * e2; Y[0][1] = xi * e2 * e3;
                        X[1][0] = xi * e2; X[1][1] = xi * e2 * e1;
                        Y[1][0] = xi; Y[1][1] = xi * e3;
                        W[0] = W[1] = jac;
                        nr = 2;
                    }
                    for (int r = 0; r < nr; ++r)
                        sum += w0 * W[r] * pow(X[r][0], a) * pow(X[r][1], b) * pow(Y[r][0], c) *
                               pow(Y[r][1], d);
                }
    return sum;
}
