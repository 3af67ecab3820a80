// Host-side data structures of libgaca (mesh, cluster tree, block partition).
#pragma once

#include <array>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace gaca {

const char *last_error();
void options_default(gaca_options *o);

struct HostMesh {
    int64_t nv = 0, M = 0;
    std::vector<double> xyz;
    std::vector<int32_t> tri;
    // per element (original order)
    std::vector<double> vert;   // 9 per element: a, b, c
    std::vector<double> cen;    // centroid
    std::vector<double> nrm;    // unit normal
    std::vector<double> area, dpl, hmax;
    std::vector<double> vmin, vmax;  // vertex box
    void init(const double *xyz, int64_t nv, const int32_t *tri, int64_t M);
};

struct ClusterTree {
    struct Node {
        int64_t start = 0, size = 0;
        int32_t level = 0;
        int32_t child[2] = {-1, -1};
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        double diam = 0.0;
    };
    int32_t leaf_size = 32;
    std::vector<int64_t> perm;   // tree position -> original id
    std::vector<Node> nodes;     // nodes[0] = root
    void build(const HostMesh &mesh, int32_t leaf);

   private:
    int32_t build_rec(const HostMesh &mesh, int64_t start, int64_t size, int level);
};

struct Partition {
    double eta = 1.0;
    std::vector<std::array<int64_t, 4>> far, near;   // (row_start, m, col_start, n)
    std::vector<int32_t> far_level;
    std::vector<std::array<int32_t, 2>> far_nodes;   // (row cluster, column cluster) node ids
    void build(const ClusterTree &tree, double eta);
};

int32_t collocation_tier(const HostMesh &mesh, int64_t i, int64_t j);
int32_t galerkin_tier(const HostMesh &mesh, int64_t i, int64_t j);
constexpr int kNumTiers = 6;          // pair classes (collocation uses the first 4)
constexpr int kGalerkinNTheta = 16;   // Gauss points per angular sector (coincident pairs)

// gCQ integration points and weights (App. A); throws Error on invalid input.
void gcq_contour(int stages, const double *rk_A, double dt_min, double dt_max, int n_q,
                 double *s_re, double *s_im, double *w_re, double *w_im);

}  // namespace gaca
