// Launch wrappers of the HIP kernels (defined in kernels.hip).
#pragma once

#include "internal.h"

namespace gaca {

struct NearPair {
    int32_t blk;
    int16_t i, j;   // tree-local row / column inside the near block
};

struct NearBlockDev {
    int32_t r0, m, c0, n;
    int64_t off;     // offset (complex elements) of the [m][L][n] block
};

// Near field: every pair of one tier, all frequencies, FP64 compute, stored as double2
// (out64) or float2 (out32).
void launch_near(int kernel, int tier, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                 const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                 double2 *out64, float2 *out32, hipStream_t st);

// Galerkin single layer near field, one pair class (GalTier) per launch.
void launch_near_galerkin(int tier, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                          const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                          double2 *out64, float2 *out32, hipStream_t st);

// Kernel ids used by the far-field and eval launches: 0 collocation single layer,
// 1 collocation double layer, 2 Galerkin single layer.
// Far field 3D-ACA: one workgroup per block of `blocks` (nb blocks).
// kind 0: small blocks (m n <= 1024, sides <= 64), residual face in LDS, 64 threads;
// kind 1: small blocks (m n <= 2304, sides <= 96), residual face in LDS, 256 threads;
// kind 2: large blocks, residual face and factors in HBM scratch, 512 threads.
// Small kinds need rcap <= 64.
struct FarLaunch {
    const FarBlockDev *blocks;
    int32_t nb;
    int32_t kind;
    int32_t mixed;        // 1: FP32 faces/factors (float2), FP64 bookkeeping
    void *scratch;        // byte offsets in FarBlockDev
    FarMeta *meta;
    CrossMeta *cmeta;     // [nfar][rcap]
    int64_t *cross_off;   // [nfar][rcap] arena offsets (elements) of U (then W follows)
    void *arena;          // double2 (FP64) or float2 (mixed) factors
    unsigned long long *arena_ctr;
    unsigned long long arena_cap;
    double2 *fib_arena;
    unsigned long long *fib_ctr;
    unsigned long long fib_cap;
    int64_t *fib_off;     // [nfar]
    int32_t *overflow;
    const double2 *dense; // synthetic-entry mode: dense tensor [m][n][L] (block 0 only)
};
void launch_far(int kernel, const GeoDev &g, const FreqDev &f, const AcaParams &P,
                     const FarLaunch &fl, hipStream_t st);

// Test hook: entries of (row, col) tree positions with given tiers at frequency k.
void launch_eval(int kernel, const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                 const int32_t *rows, const int32_t *cols, const int32_t *ks,
                 const int32_t *tiers, double2 *out, hipStream_t st);

// Apply (FP64, VALU reference path).
struct ApplyDev {
    int32_t L, nrhs;
    int64_t M;
    const int64_t *perm;          // tree pos -> original id
    int32_t nfar, nnear, rcap;
    const int32_t *far4;          // [nfar][4]
    const FarMeta *meta;
    const CrossMeta *cmeta;
    const int64_t *cross_off;
    const void *arena;            // double2 (FP64 build) or float2 (mixed build) factors
    int32_t fac_fp32;
    const int64_t *fib_off;
    const double2 *fib_arena;
    const NearBlockDev *nblocks;
    const double2 *near64;
    const float2 *near32;
    // leaf CSR: leaf -> covering far blocks / near blocks
    int32_t nleaf;
    const int32_t *leaf_r0, *leaf_m;
    const int32_t *leaf_far_ptr, *leaf_far_idx;
    const int32_t *leaf_near_ptr, *leaf_near_idx;
    const int64_t *z_off;         // [nfar] offset of the block's z (sum_rho x nrhs) or v
};
// x_fp32: X, Y and the workspace are complex64 (FP32 arithmetic), else complex128.
// Workspace pointers are in elements of that type.
void launch_apply(const ApplyDev &a, int mode, int x_fp32, const void *X, void *Y, void *Xp,
                  void *Yp, void *zbuf, void *tbuf, const int64_t *t_off, void *ybuf,
                  const int64_t *y_off, hipStream_t st);

}  // namespace gaca
