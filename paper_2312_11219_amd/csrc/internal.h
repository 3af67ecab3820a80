// Internal types shared by the host code and the HIP kernels of libgaca.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gaca.h"

namespace gaca {

// ---- error state ---------------------------------------------------------------------
void set_error(const std::string &msg);
struct Error {
    gaca_status code;
    std::string msg;
};

#define GACA_HIP_CHECK(expr)                                                              \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::gaca::Error{GACA_ERR_HIP, std::string(#expr) + ": " +                 \
                                                  hipGetErrorString(e_)};                 \
    } while (0)

// ---- quadrature tables (host generated, independent derivations) ---------------------
struct Rule1D {
    std::vector<double> x, w;   // nodes / weights on [0, 1]
};
Rule1D gauss_legendre01(int n);
// Symmetric 6-point degree-4 triangle rule: barycentric (6 x 3) and weights summing to 1.
void triangle6(double bary[6][3], double w[6]);

// ---- device views ----------------------------------------------------------------------
// Geometry in tree order, structure of arrays (length M each).
struct GeoDev {
    int64_t M;
    const double *ax, *ay, *az, *bx, *by, *bz, *cx, *cy, *cz;  // vertices
    const double *xx, *xy, *xz;                                // centroids (collocation points)
    const double *nx, *ny, *nz, *d;                            // unit normal, plane offset n.a
    const double *h, *area;                                    // longest edge, area
    const double *q6x, *q6y, *q6z, *q6w;                       // [6][M] far-rule points/weights
    // FP32 copies for the mixed-precision far field: far-rule points relative to the
    // element centroid (small, so FP32 keeps them to ~1e-7 of the element size) and weights
    const float *q6dx, *q6dy, *q6dz, *q6wf;                    // [6][M]
    // P1 double layer collocated at the vertices (scheme GACA_COLLOCATION_P1): the degrees
    // of freedom are the M vertices (tree order; xx, xy, xz hold their coordinates); the
    // triangle arrays (ax .. area, q6x/y/z as [6][T]) are indexed by triangle id in the
    // original order, tcx/tcy/tcz their centroids; the patch of the vertex at tree position j
    // is ptri / ploc[pptr[j] .. pptr[j + 1]) (triangle id, local index of the vertex in it);
    // tv0/tv1/tv2 are the vertex ids of each triangle, dvid the vertex id of each tree
    // position; q6wl[(loc 6 + p) T + t] = weight x area x barycentric coordinate loc of rule
    // point p.  For the other schemes T = M and the P1 pointers are null.
    int64_t T;
    const int32_t *pptr, *ptri, *ploc, *tv0, *tv1, *tv2, *dvid;
    const double *tcx, *tcy, *tcz, *q6wl;
};

// Quadrature tables in device memory.
struct QuadDev {
    int n4, n8, nd, ng, ns;
    const double *g4;    // n4 x 2 (node, weight)
    const double *g8;    // n8 x 2
    const double *gd;    // nd x 2
    const double *gg;    // ng x 2 (Galerkin disjoint pairs with q < 2)
    const double *gs;    // ns x 2 (Galerkin pairs sharing an edge or a vertex)
    const double *r6;    // 6 x 4 (bary, weight)
    int nth;
    const double *gth;   // nth x 2 (Galerkin coincident pairs, per angular sector)
};

struct FreqDev {
    int L;
    int L_eval;          // frequencies actually evaluated (L or ceil(L/2) with mirror)
    int mirror;          // 1: s_{L-1-l} = conj(s_l) exactly
    const double *re, *im;
};

enum Tier : int32_t { TIER_FAR6 = 0, TIER_MID4 = 1, TIER_NEAR8 = 2, TIER_SELF = 3 };

// One admissible block of a far-field batch (constant during the build).
struct FarBlockDev {
    int32_t r0, m, c0, n;      // tree-order ranges
    int64_t uw_off;            // face-type elements: this block's U (rho_max x m) then W (rho_max x n)
    int32_t rho_max;           // face-rank cap for this block
    int32_t out_idx;           // global far-block index
    // mixed-precision scaling, c_k = exp(-s_k d0f): with D = x_sigma - y_tau (box centres),
    // Dh = fl32(D), d0f = fl32(|D|), kappa = |Dh|^2 - d0f^2 (exact in FP64) and
    // xs_adj = x_sigma - (D - Dh) (so row offsets absorb the rounding of D)
    double xs_adj[3], yt[3];
    float Dh[3], d0f, kappa;
    int32_t kern;              // kernel id of the block's operator (joint builds mix 0 and 1)
    int32_t which;             // operator index of a joint build (0 or 1)
    int32_t pad_;
};

// Mutable 3D-ACA state of one far block between the phases of an iteration.
struct FarStateDev {
    int32_t ell, k, zero_run, zero_faces, capped, sum_rho, nused_k, done;
    int32_t rho;               // rank of the current face (0: zero face)
    int32_t pidx;              // pivot of the current face (row-major index), small blocks
    double norm2, scale;       // ||C^(l)||_F^2 and max_p |H_p[i_p, j_p]| max_k |f_p[k]|
    double ref2, zero_tol;     // current face: ||C^(l-1)(:,:,k)||^2 (face frame), zero threshold
    double mxh, h2;            // current face: max |H_l|^2 and ||H_l||_F^2, small blocks
    int64_t aca_ticks;         // device wall-clock ticks spent in the face ACAs so far
};

// Per-block result metadata written by the far-field kernel.
struct FarMeta {
    int32_t rank;              // crosses
    int32_t sum_rho;
    int32_t capped;
    int32_t zero_faces;
    int64_t aca_ticks;         // device wall-clock ticks of the block's face ACAs (sum)
    double norm2;
};

struct CrossMeta {
    int32_t k, pi, pj, rho;
};

struct AcaParams {
    double eps, eps_aca, tie, delta;
    int32_t rcap;              // crosses per block
    int32_t kernel;            // 0 SLP, 1 DLP
    int32_t galerkin;          // 1 Galerkin
    int32_t zero_batch;        // several rows per pass in the large-face zero-row search
    int32_t recompress;        // faces recompressed after their ACA
    int32_t pivot_index;       // pivot by the eq. (index) row estimate
};

}  // namespace gaca
