/*
 * Oracle: integrated kernel entries E(i, j, k) of the Laplace-domain single and double
 * layer on flat triangles with piecewise-constant (P0) functions.
 *
 * TEST INFRASTRUCTURE ONLY -- plain FP64 loops, no blocking, no reordering; called from
 * Python through ctypes by oracle/entries.py.  Shares no code with the GPU library.
 *
 * Definition (paper Sec. 2 and Sec. 3):
 *   Laplace-domain fundamental solution with wave speed c = 1:
 *       G_s(r) = exp(-s r) / (4 pi r),
 *   double layer kernel (normal derivative in y, outward normal n_y):
 *       dG/dn_y = exp(-s r) (1 + s r) ((x - y) . n_y) / (4 pi r^3),
 *   and for y in the plane of triangle j, (x - y) . n_j = n_j . x - d_j with d_j = n_j . a_j.
 *   Collocation P0 (eq. bie_semi_diri, collocation point read as the centroid x_i):
 *       V_ij(s) = int_{tau_j} G_s(|x_i - y|) dS_y,  K_ij(s) = int_{tau_j} dG/dn_y dS_y.
 *
 * Quadrature (the paper's distance heuristic is unspecified; this reading fixes it):
 *   q = |x_i - x_j| / h_j, h_j the longest edge of triangle j;
 *   entries of admissible (far) blocks: 6-point rule;
 *   near blocks: i == j -> three Duffy-mapped sub-triangles split at x_i, n_D x n_D Gauss
 *                (n_D = 16 by default);
 *                q >= 4 -> 6-point rule; 2 <= q < 4 -> collapsed 4x4; q < 2 -> collapsed 8x8.
 *   The double layer self entry is 0 (x_i lies in the plane of its own flat triangle).
 *
 * Parity pins: tests/test_oracle_entries.py (closed forms on the unit sphere, Gauss
 * solid-angle identity, 1-D angular formula for the self term, convergence in order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define PI 3.14159265358979323846

typedef struct {
    double a[3], b[3], c[3];
    double x[3];     /* centroid */
    double n[3];     /* unit normal */
    double area, d, h;
} tri_t;

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

static void make_tri(const double *v9, tri_t *t) {
    double e1[3], e2[3], e3[3], nn[3];
    for (int k = 0; k < 3; ++k) {
        t->a[k] = v9[k];
        t->b[k] = v9[3 + k];
        t->c[k] = v9[6 + k];
        t->x[k] = (t->a[k] + t->b[k] + t->c[k]) / 3.0;
    }
    sub3(t->b, t->a, e1);
    sub3(t->c, t->a, e2);
    cross3(e1, e2, nn);
    double len = norm3(nn);
    t->area = 0.5 * len;
    for (int k = 0; k < 3; ++k) t->n[k] = nn[k] / len;
    t->d = dot3(t->n, t->a);
    sub3(t->c, t->b, e3);
    double h = norm3(e1), h2 = norm3(e2), h3 = norm3(e3);
    if (h2 > h) h = h2;
    if (h3 > h) h = h3;
    t->h = h;
}

/* Quadrature point list for one entry: positions and weights (weights include the
 * surface Jacobian, so sum(w) = area of the integration domain). */
typedef struct {
    int n;
    double *y;   /* 3 * n */
    double *w;   /* n */
} qlist_t;

typedef struct {
    const double *r6;   /* 6 x 4: l1, l2, l3, weight (weights sum to 1) */
    int n4; const double *g4;   /* n4 x 2: node, weight on [0,1] */
    int n8; const double *g8;
    int nd; const double *gd;
} rules_t;

static void push(qlist_t *q, const double *y, double w) {
    q->y[3 * q->n] = y[0];
    q->y[3 * q->n + 1] = y[1];
    q->y[3 * q->n + 2] = y[2];
    q->w[q->n] = w;
    q->n++;
}

static void rule6_points(const tri_t *t, const rules_t *R, qlist_t *q) {
    for (int p = 0; p < 6; ++p) {
        const double *r = R->r6 + 4 * p;
        double y[3];
        for (int k = 0; k < 3; ++k) y[k] = r[0] * t->a[k] + r[1] * t->b[k] + r[2] * t->c[k];
        push(q, y, r[3] * t->area);
    }
}

/* Collapsed n x n rule on triangle (a, b, c), edge u = 0 collapsed onto vertex a:
 * y = a + u (b - a) + u v (c - b),  dS = |(b - a) x (c - b)| u du dv. */
static void collapsed_points(const double *a, const double *b, const double *c,
                             int n, const double *g, qlist_t *q) {
    double e1[3], e2[3], nn[3];
    sub3(b, a, e1);
    sub3(c, b, e2);
    cross3(e1, e2, nn);
    double two_area = norm3(nn);
    for (int iu = 0; iu < n; ++iu) {
        double u = g[2 * iu], wu = g[2 * iu + 1];
        for (int iv = 0; iv < n; ++iv) {
            double v = g[2 * iv], wv = g[2 * iv + 1];
            double y[3];
            for (int k = 0; k < 3; ++k) y[k] = a[k] + u * e1[k] + u * v * e2[k];
            push(q, y, wu * wv * u * two_area);
        }
    }
}

/* Collocation self term: split the triangle at x into (x,b,c), (x,c,a), (x,a,b) and
 * apply the collapsed rule with the collapsed vertex at x (Duffy transformation). */
static void self_points(const tri_t *t, const rules_t *R, qlist_t *q) {
    collapsed_points(t->x, t->b, t->c, R->nd, R->gd, q);
    collapsed_points(t->x, t->c, t->a, R->nd, R->gd, q);
    collapsed_points(t->x, t->a, t->b, R->nd, R->gd, q);
}

/* Sum over the quadrature list of the kernel at every frequency.
 * kernel 0: single layer, 1: double layer. */
static void integrate(int kernel, const double *x, const tri_t *tj, const qlist_t *q,
                      int L, const double *s_re, const double *s_im, double *out) {
    double num = 0.0;
    if (kernel == 1) num = dot3(tj->n, x) - tj->d;
    for (int l = 0; l < L; ++l) {
        double acc_re = 0.0, acc_im = 0.0;
        for (int p = 0; p < q->n; ++p) {
            double dv[3];
            sub3(x, q->y + 3 * p, dv);
            double r = norm3(dv);
            /* exp(-s r) = exp(-Re(s) r) (cos(Im(s) r) - i sin(Im(s) r)) */
            double mag = exp(-s_re[l] * r);
            double e_re = mag * cos(s_im[l] * r);
            double e_im = -mag * sin(s_im[l] * r);
            double g_re, g_im;
            if (kernel == 0) {
                g_re = e_re / (4.0 * PI * r);
                g_im = e_im / (4.0 * PI * r);
            } else {
                /* exp(-s r) (1 + s r) / (4 pi r^3) */
                double f_re = 1.0 + s_re[l] * r, f_im = s_im[l] * r;
                double p_re = e_re * f_re - e_im * f_im;
                double p_im = e_re * f_im + e_im * f_re;
                double den = 4.0 * PI * r * r * r;
                g_re = p_re / den;
                g_im = p_im / den;
            }
            acc_re += q->w[p] * g_re;
            acc_im += q->w[p] * g_im;
        }
        if (kernel == 1) {
            acc_re *= num;
            acc_im *= num;
        }
        out[2 * l] = acc_re;
        out[2 * l + 1] = acc_im;
    }
}

/* Tier codes returned to the caller for statistics. */
enum { TIER_FAR6 = 0, TIER_MID4 = 1, TIER_NEAR8 = 2, TIER_SELF = 3 };

/*
 * Collocation entries for a list of (row, col) element pairs at all L frequencies.
 *   tri9:  M x 9 vertex coordinates (a, b, c) per element
 *   ii,jj: element ids (same numbering as tri9), far: 1 if the pair lies in an
 *          admissible block (always the 6-point rule)
 *   out:   npair x L x 2 (re, im);  tier_out (optional): tier code per pair
 */
void oracle_collocation_entries(int kernel, int64_t M, const double *tri9,
                                int L, const double *s_re, const double *s_im,
                                int64_t npair, const int64_t *ii, const int64_t *jj,
                                const int32_t *far,
                                const double *r6, int n4, const double *g4,
                                int n8, const double *g8, int nd, const double *gd,
                                double *out, int32_t *tier_out) {
    (void)M;
    rules_t R = {r6, n4, g4, n8, g8, nd, gd};
    int maxq = 3 * nd * nd;
    if (n8 * n8 > maxq) maxq = n8 * n8;
    if (n4 * n4 > maxq) maxq = n4 * n4;
    if (6 > maxq) maxq = 6;
#pragma omp parallel
    {
        qlist_t q;
        q.y = (double *)malloc(sizeof(double) * 3 * maxq);
        q.w = (double *)malloc(sizeof(double) * maxq);
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < npair; ++p) {
            tri_t ti, tj;
            make_tri(tri9 + 9 * ii[p], &ti);
            make_tri(tri9 + 9 * jj[p], &tj);
            q.n = 0;
            int tier;
            if (ii[p] == jj[p]) {
                tier = TIER_SELF;
            } else if (far[p]) {
                tier = TIER_FAR6;
            } else {
                double dv[3];
                sub3(ti.x, tj.x, dv);
                double qd = norm3(dv) / tj.h;
                tier = qd >= 4.0 ? TIER_FAR6 : (qd >= 2.0 ? TIER_MID4 : TIER_NEAR8);
            }
            if (tier_out) tier_out[p] = tier;
            double *o = out + 2 * (size_t)L * p;
            if (tier == TIER_SELF && kernel == 1) {
                for (int l = 0; l < 2 * L; ++l) o[l] = 0.0;
                continue;
            }
            switch (tier) {
                case TIER_SELF: self_points(&tj, &R, &q); break;
                case TIER_FAR6: rule6_points(&tj, &R, &q); break;
                case TIER_MID4: collapsed_points(tj.a, tj.b, tj.c, n4, g4, &q); break;
                default: collapsed_points(tj.a, tj.b, tj.c, n8, g8, &q); break;
            }
            integrate(kernel, ti.x, &tj, &q, L, s_re, s_im, o);
        }
        free(q.y);
        free(q.w);
    }
}

/*
 * Collocation entries with an explicit collapsed n x n rule (or the self split for i == j)
 * on every pair, used to measure each tier's quadrature error against a much higher order.
 */
void oracle_collocation_entries_order(int kernel, const double *tri9, int L,
                                      const double *s_re, const double *s_im, int64_t npair,
                                      const int64_t *ii, const int64_t *jj, int n,
                                      const double *g, double *out) {
#pragma omp parallel
    {
        qlist_t q;
        q.y = (double *)malloc(sizeof(double) * 3 * 3 * n * n);
        q.w = (double *)malloc(sizeof(double) * 3 * n * n);
        rules_t R = {0, 0, 0, 0, 0, n, g};
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npair; ++p) {
            tri_t ti, tj;
            make_tri(tri9 + 9 * ii[p], &ti);
            make_tri(tri9 + 9 * jj[p], &tj);
            q.n = 0;
            double *o = out + 2 * (size_t)L * p;
            if (ii[p] == jj[p]) {
                if (kernel == 1) {
                    for (int l = 0; l < 2 * L; ++l) o[l] = 0.0;
                    continue;
                }
                self_points(&tj, &R, &q);
            } else {
                collapsed_points(tj.a, tj.b, tj.c, n, g, &q);
            }
            integrate(kernel, ti.x, &tj, &q, L, s_re, s_im, o);
        }
        free(q.y);
        free(q.w);
    }
}

/* ------------------------------------------------------------------------------------
 * P1 double layer, collocation at the mesh vertices (eq. bie_semi_diri with the trial
 * functions phi_j linear continuous, the collocation points x_i at the nodes):
 *   K_ij(s) = sum over the triangles tau of supp phi_j of
 *             int_tau dG/dn_y(x_i - y) lambda_{tau,j}(y) dS_y,
 * lambda_{tau,j} = phi_j on tau = the barycentric coordinate of vertex j in tau.
 * Per (x_i, tau): a triangle with x_i among its vertices contributes exactly 0 (x_i lies in
 * its plane, so (x_i - y) . n_tau = 0 on it); otherwise far pairs take the 6-point rule and
 * near pairs the tier of q = |x_i - c_tau| / h_tau (q >= 4: 6-point, 2 <= q < 4: collapsed
 * 4 x 4, q < 2: collapsed 8 x 8), the collapsed rules with the collapsed edge at the first
 * vertex of tau, on which lambda = (1 - u, u (1 - v), u v).
 * ------------------------------------------------------------------------------------ */

static void rule6_points_p1(const tri_t *t, const rules_t *R, int loc, qlist_t *q) {
    for (int p = 0; p < 6; ++p) {
        const double *r = R->r6 + 4 * p;
        double y[3];
        for (int k = 0; k < 3; ++k) y[k] = r[0] * t->a[k] + r[1] * t->b[k] + r[2] * t->c[k];
        push(q, y, r[3] * t->area * r[loc]);
    }
}

static void collapsed_points_p1(const tri_t *t, int n, const double *g, int loc, qlist_t *q) {
    double e1[3], e2[3], nn[3];
    sub3(t->b, t->a, e1);
    sub3(t->c, t->b, e2);
    cross3(e1, e2, nn);
    double two_area = norm3(nn);
    for (int iu = 0; iu < n; ++iu) {
        double u = g[2 * iu], wu = g[2 * iu + 1];
        for (int iv = 0; iv < n; ++iv) {
            double v = g[2 * iv], wv = g[2 * iv + 1];
            double lam = loc == 0 ? 1.0 - u : (loc == 1 ? u * (1.0 - v) : u * v);
            double y[3];
            for (int k = 0; k < 3; ++k) y[k] = t->a[k] + u * e1[k] + u * v * e2[k];
            push(q, y, wu * wv * u * two_area * lam);
        }
    }
}

/*
 *   xyz:  nv x 3 vertex coordinates;  tri: ntri x 3 vertex ids (counter-clockwise seen
 *         from outside);  pptr (nv + 1), ptri, ploc: the triangles of each vertex's patch
 *         and the vertex's local index (0, 1, 2) in each
 *   ii, jj: vertex ids; far: 1 if the pair lies in an admissible block
 *   order > 0: every non-zero (x_i, tau) with the collapsed order x order rule instead
 *   out: npair x L x 2
 */
void oracle_p1_dlp_entries(const double *xyz, const int32_t *tri, const int64_t *pptr,
                           const int32_t *ptri, const int32_t *ploc, int L,
                           const double *s_re, const double *s_im, int64_t npair,
                           const int64_t *ii, const int64_t *jj, const int32_t *far,
                           const double *r6, int n4, const double *g4, int n8,
                           const double *g8, int order, const double *go, double *out) {
    rules_t R = {r6, n4, g4, n8, g8, 0, 0};
    int maxq = 6;
    if (n4 * n4 > maxq) maxq = n4 * n4;
    if (n8 * n8 > maxq) maxq = n8 * n8;
    if (order * order > maxq) maxq = order * order;
#pragma omp parallel
    {
        qlist_t q;
        q.y = (double *)malloc(sizeof(double) * 3 * maxq);
        q.w = (double *)malloc(sizeof(double) * maxq);
        double *tmp = (double *)malloc(sizeof(double) * 2 * L);
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < npair; ++p) {
            const double *x = xyz + 3 * ii[p];
            double *o = out + 2 * (size_t)L * p;
            for (int l = 0; l < 2 * L; ++l) o[l] = 0.0;
            for (int64_t e = pptr[jj[p]]; e < pptr[jj[p] + 1]; ++e) {
                const int32_t *tv = tri + 3 * (int64_t)ptri[e];
                if (tv[0] == ii[p] || tv[1] == ii[p] || tv[2] == ii[p]) continue;
                double v9[9];
                for (int c = 0; c < 3; ++c)
                    for (int k = 0; k < 3; ++k) v9[3 * c + k] = xyz[3 * (int64_t)tv[c] + k];
                tri_t t;
                make_tri(v9, &t);
                q.n = 0;
                const int loc = ploc[e];
                if (order > 0) {
                    collapsed_points_p1(&t, order, go, loc, &q);
                } else if (far[p]) {
                    rule6_points_p1(&t, &R, loc, &q);
                } else {
                    double dv[3];
                    sub3(x, t.x, dv);
                    double qd = norm3(dv) / t.h;
                    if (qd >= 4.0) rule6_points_p1(&t, &R, loc, &q);
                    else if (qd >= 2.0) collapsed_points_p1(&t, n4, g4, loc, &q);
                    else collapsed_points_p1(&t, n8, g8, loc, &q);
                }
                integrate(1, x, &t, &q, L, s_re, s_im, tmp);
                for (int l = 0; l < 2 * L; ++l) o[l] += tmp[l];
            }
        }
        free(q.y);
        free(q.w);
        free(tmp);
    }
}
