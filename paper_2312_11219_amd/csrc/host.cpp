// Host-side logic of libgaca: error state, options, quadrature tables, geometry in
// structure-of-arrays form, cluster tree and block partition (Sec. 4 of the paper:
// balanced cluster tree, purely geometric admissibility, the same partition for every
// frequency).  Compiled with -ffp-contract=off so that every geometric decision (median
// order, admissibility, quadrature tier) is taken with plain IEEE operations.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace gaca {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

void options_default(gaca_options *o) {
    std::memset(o, 0, sizeof(*o));
    o->leaf_size = 32;
    o->eta = 1.0;
    o->eps3d = 1e-6;
    o->eps_aca = 1e-8;
    o->precision = GACA_FP64;
    o->quad_mid = 4;
    o->quad_near = 8;
    o->n_duffy = 16;
    o->n_galerkin = 5;
    o->n_touch = 12;
    o->tie = 1e-9;
    o->delta_zero = 1e-13;
    o->max_rank3d = 64;
    o->max_face_rank = 0;
    o->max_device_bytes = 0;
    o->batch_bytes = 160ull << 30;
    o->threads_small = 128;
    o->threads_large = 0;
    o->verbose = 0;
    o->zero_rows_batch = 1;
    o->autotune_cache = nullptr;
}

// ---- Gauss-Legendre on [0, 1] by Newton iteration on the Legendre recurrence ----------
Rule1D gauss_legendre01(int n) {
    Rule1D r;
    r.x.resize(n);
    r.w.resize(n);
    for (int i = 0; i < n; ++i) {
        // Chebyshev-like initial guess for the i-th root of P_n on [-1, 1] (descending)
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            double pn = (n == 0) ? 1.0 : (n == 1 ? t : p1);
            double pnm1 = (n == 1) ? 1.0 : p0;
            dp = n * (t * pn - pnm1) / (t * t - 1.0);
            double dt = pn / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) {
                // one more evaluation for the derivative at the converged root
                p0 = 1.0;
                p1 = t;
                for (int k = 2; k <= n; ++k) {
                    double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = pk;
                }
                pn = (n == 1) ? t : p1;
                pnm1 = (n == 1) ? 1.0 : p0;
                dp = n * (t * pn - pnm1) / (t * t - 1.0);
                break;
            }
        }
        double w = 2.0 / ((1.0 - t * t) * dp * dp);
        // map to [0, 1], ascending order
        r.x[n - 1 - i] = 0.5 * (t + 1.0);
        r.w[n - 1 - i] = 0.5 * w;
    }
    return r;
}

// ---- symmetric 6-point degree-4 triangle rule ---------------------------------------
// Two orbits (a, a, 1 - 2a) with three points each; exactness for the symmetric
// invariants 1, e2, e3, e2^2 (e2 = sum l_i l_j, e3 = l1 l2 l3) over the triangle, whose
// area averages are 1, 1/4, 1/60, 1/15, gives four equations solved by Newton.
void triangle6(double bary[6][3], double w[6]) {
    double a1 = 0.44, a2 = 0.09, w1 = 0.22, w2 = 0.11;
    auto e2 = [](double a) { return 2.0 * a - 3.0 * a * a; };
    auto e3 = [](double a) { return a * a * (1.0 - 2.0 * a); };
    auto de2 = [](double a) { return 2.0 - 6.0 * a; };
    auto de3 = [](double a) { return 2.0 * a - 6.0 * a * a; };
    for (int it = 0; it < 100; ++it) {
        double F[4] = {3 * w1 + 3 * w2 - 1.0, 3 * w1 * e2(a1) + 3 * w2 * e2(a2) - 0.25,
                       3 * w1 * e3(a1) + 3 * w2 * e3(a2) - 1.0 / 60.0,
                       3 * w1 * e2(a1) * e2(a1) + 3 * w2 * e2(a2) * e2(a2) - 1.0 / 15.0};
        // Jacobian w.r.t. (a1, a2, w1, w2)
        double J[4][4] = {{0, 0, 3, 3},
                          {3 * w1 * de2(a1), 3 * w2 * de2(a2), 3 * e2(a1), 3 * e2(a2)},
                          {3 * w1 * de3(a1), 3 * w2 * de3(a2), 3 * e3(a1), 3 * e3(a2)},
                          {6 * w1 * e2(a1) * de2(a1), 6 * w2 * e2(a2) * de2(a2),
                           3 * e2(a1) * e2(a1), 3 * e2(a2) * e2(a2)}};
        // solve J dx = F by Gaussian elimination with partial pivoting
        double A[4][5];
        for (int r = 0; r < 4; ++r) {
            for (int c = 0; c < 4; ++c) A[r][c] = J[r][c];
            A[r][4] = F[r];
        }
        for (int c = 0; c < 4; ++c) {
            int piv = c;
            for (int r = c + 1; r < 4; ++r)
                if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
            for (int k = 0; k < 5; ++k) std::swap(A[c][k], A[piv][k]);
            for (int r = c + 1; r < 4; ++r) {
                double f = A[r][c] / A[c][c];
                for (int k = c; k < 5; ++k) A[r][k] -= f * A[c][k];
            }
        }
        double dx[4];
        for (int r = 3; r >= 0; --r) {
            double s = A[r][4];
            for (int k = r + 1; k < 4; ++k) s -= A[r][k] * dx[k];
            dx[r] = s / A[r][r];
        }
        a1 -= dx[0];
        a2 -= dx[1];
        w1 -= dx[2];
        w2 -= dx[3];
        if (std::fabs(dx[0]) + std::fabs(dx[1]) + std::fabs(dx[2]) + std::fabs(dx[3]) < 1e-17)
            break;
    }
    const double as[2] = {a1, a2}, ws[2] = {w1, w2};
    int p = 0;
    for (int o = 0; o < 2; ++o) {
        double a = as[o], b = 1.0 - 2.0 * a;
        const double pts[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
        for (int k = 0; k < 3; ++k, ++p) {
            bary[p][0] = pts[k][0];
            bary[p][1] = pts[k][1];
            bary[p][2] = pts[k][2];
            w[p] = ws[o];
        }
    }
}

// ---- geometry ------------------------------------------------------------------------
static inline double dot3(const double *p, const double *q) {
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
}

void HostMesh::init(const double *xyz_, int64_t nv_, const int32_t *tri_, int64_t M_) {
    if (!xyz_ || !tri_ || nv_ < 3 || M_ < 1)
        throw Error{GACA_ERR_INVALID_ARG, "mesh: null pointer or empty mesh"};
    nv = nv_;
    M = M_;
    xyz.assign(xyz_, xyz_ + 3 * nv);
    tri.assign(tri_, tri_ + 3 * M);
    for (int64_t v = 0; v < 3 * nv; ++v)
        if (!std::isfinite(xyz[v])) throw Error{GACA_ERR_INVALID_ARG, "mesh: non-finite vertex"};
    vert.resize(9 * M);
    cen.resize(3 * M);
    nrm.resize(3 * M);
    area.resize(M);
    dpl.resize(M);
    hmax.resize(M);
    vmin.resize(3 * M);
    vmax.resize(3 * M);
    for (int64_t e = 0; e < M; ++e) {
        for (int k = 0; k < 3; ++k) {
            int32_t id = tri[3 * e + k];
            if (id < 0 || id >= nv) throw Error{GACA_ERR_INVALID_ARG, "mesh: vertex id out of range"};
        }
        const double *a = &xyz[3 * tri[3 * e]];
        const double *b = &xyz[3 * tri[3 * e + 1]];
        const double *c = &xyz[3 * tri[3 * e + 2]];
        double e1[3], e2[3], e3[3], nn[3];
        for (int k = 0; k < 3; ++k) {
            vert[9 * e + k] = a[k];
            vert[9 * e + 3 + k] = b[k];
            vert[9 * e + 6 + k] = c[k];
            cen[3 * e + k] = (a[k] + b[k] + c[k]) / 3.0;
            vmin[3 * e + k] = std::min(std::min(a[k], b[k]), c[k]);
            vmax[3 * e + k] = std::max(std::max(a[k], b[k]), c[k]);
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
            e3[k] = c[k] - b[k];
        }
        nn[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nn[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nn[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double len = std::sqrt(dot3(nn, nn));
        if (!(len > 0.0)) throw Error{GACA_ERR_INVALID_ARG, "mesh: degenerate triangle"};
        area[e] = 0.5 * len;
        for (int k = 0; k < 3; ++k) nrm[3 * e + k] = nn[k] / len;
        dpl[e] = dot3(&nrm[3 * e], a);
        double h = std::sqrt(dot3(e1, e1)), h2 = std::sqrt(dot3(e2, e2)),
               h3 = std::sqrt(dot3(e3, e3));
        if (h2 > h) h = h2;
        if (h3 > h) h = h3;
        hmax[e] = h;
    }
}

// ---- cluster tree ----------------------------------------------------------------------
// Split along the longest axis of the centroid box (ties: lowest axis) at the median of
// the order (coordinate, element id); left child = first floor(n/2).
int32_t ClusterTree::build_rec(const HostMesh &mesh, int64_t start, int64_t size, int level) {
    int32_t id = (int32_t)nodes.size();
    nodes.push_back(Node{});
    Node nd;
    nd.start = start;
    nd.size = size;
    nd.level = level;
    for (int k = 0; k < 3; ++k) {
        nd.lo[k] = mesh.vmin[3 * perm[start] + k];
        nd.hi[k] = mesh.vmax[3 * perm[start] + k];
    }
    for (int64_t p = start; p < start + size; ++p) {
        int64_t e = perm[p];
        for (int k = 0; k < 3; ++k) {
            nd.lo[k] = std::min(nd.lo[k], mesh.vmin[3 * e + k]);
            nd.hi[k] = std::max(nd.hi[k], mesh.vmax[3 * e + k]);
        }
    }
    double dx = nd.hi[0] - nd.lo[0], dy = nd.hi[1] - nd.lo[1], dz = nd.hi[2] - nd.lo[2];
    nd.diam = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (size > leaf_size) {
        double cmin[3], cmax[3];
        for (int k = 0; k < 3; ++k) {
            cmin[k] = mesh.cen[3 * perm[start] + k];
            cmax[k] = cmin[k];
        }
        for (int64_t p = start; p < start + size; ++p) {
            int64_t e = perm[p];
            for (int k = 0; k < 3; ++k) {
                cmin[k] = std::min(cmin[k], mesh.cen[3 * e + k]);
                cmax[k] = std::max(cmax[k], mesh.cen[3 * e + k]);
            }
        }
        int axis = 0;
        double ext[3] = {cmax[0] - cmin[0], cmax[1] - cmin[1], cmax[2] - cmin[2]};
        for (int k = 1; k < 3; ++k)
            if (ext[k] > ext[axis]) axis = k;
        std::sort(perm.begin() + start, perm.begin() + start + size,
                  [&](int64_t a, int64_t b) {
                      double ca = mesh.cen[3 * a + axis], cb = mesh.cen[3 * b + axis];
                      if (ca != cb) return ca < cb;
                      return a < b;
                  });
        int64_t half = size / 2;
        nd.child[0] = build_rec(mesh, start, half, level + 1);
        nd.child[1] = build_rec(mesh, start + half, size - half, level + 1);
    }
    nodes[id] = nd;
    return id;
}

void ClusterTree::build(const HostMesh &mesh, int32_t leaf) {
    if (leaf < 1) throw Error{GACA_ERR_INVALID_ARG, "leaf_size must be >= 1"};
    leaf_size = leaf;
    perm.resize(mesh.M);
    std::iota(perm.begin(), perm.end(), 0);
    nodes.clear();
    nodes.reserve(4 * (mesh.M / std::max<int64_t>(1, leaf)) + 8);
    build_rec(mesh, 0, mesh.M, 0);
}

static bool admissible(const ClusterTree::Node &s, const ClusterTree::Node &t, double eta) {
    double g[3];
    for (int k = 0; k < 3; ++k) {
        double a = s.lo[k] - t.hi[k], b = t.lo[k] - s.hi[k];
        g[k] = std::max(0.0, std::max(a, b));
    }
    double dist = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    return dist > 0.0 && std::min(s.diam, t.diam) <= eta * dist;
}

void Partition::build(const ClusterTree &tree, double eta_) {
    eta = eta_;
    far.clear();
    near.clear();
    far_level.clear();
    far_nodes.clear();
    struct Pair {
        int32_t s, t;
    };
    // explicit stack, pushing children in reverse so the order matches the recursion
    // (s1,t1), (s1,t2), (s2,t1), (s2,t2)
    std::vector<Pair> stack{{0, 0}};
    while (!stack.empty()) {
        Pair pr = stack.back();
        stack.pop_back();
        const auto &s = tree.nodes[pr.s];
        const auto &t = tree.nodes[pr.t];
        if (admissible(s, t, eta)) {
            far.push_back({s.start, s.size, t.start, t.size});
            far_level.push_back(std::max(s.level, t.level));
            far_nodes.push_back({pr.s, pr.t});
        } else if (s.child[0] < 0 || t.child[0] < 0) {
            near.push_back({s.start, s.size, t.start, t.size});
        } else {
            for (int a = 1; a >= 0; --a)
                for (int b = 1; b >= 0; --b) stack.push_back({s.child[a], t.child[b]});
        }
    }
}

// Quadrature tier of a near-block collocation pair (i, j) in ORIGINAL ids:
// q = |x_i - x_j| / h_j.
int32_t collocation_tier(const HostMesh &mesh, int64_t i, int64_t j) {
    if (i == j) return TIER_SELF;
    double dv[3];
    for (int k = 0; k < 3; ++k) dv[k] = mesh.cen[3 * i + k] - mesh.cen[3 * j + k];
    double q = std::sqrt(dot3(dv, dv)) / mesh.hmax[j];
    return q >= 4.0 ? TIER_FAR6 : (q >= 2.0 ? TIER_MID4 : TIER_NEAR8);
}

// Galerkin pair class in ORIGINAL ids: 5 coincident, 3 common edge, 4 common vertex, else
// by q = |x_i - x_j| / max(h_i, h_j): 0 (q >= 4), 1 (2 <= q < 4), 2 (q < 2).
int32_t galerkin_tier(const HostMesh &mesh, int64_t i, int64_t j) {
    if (i == j) return 5;
    int shared = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (mesh.tri[3 * i + a] == mesh.tri[3 * j + b]) ++shared;
    if (shared >= 2) return 3;
    if (shared == 1) return 4;
    double dv[3];
    for (int k = 0; k < 3; ++k) dv[k] = mesh.cen[3 * i + k] - mesh.cen[3 * j + k];
    const double hm = mesh.hmax[i] > mesh.hmax[j] ? mesh.hmax[i] : mesh.hmax[j];
    const double q = std::sqrt(dot3(dv, dv)) / hm;
    return q >= 4.0 ? 0 : (q >= 2.0 ? 1 : 2);
}

}  // namespace gaca
