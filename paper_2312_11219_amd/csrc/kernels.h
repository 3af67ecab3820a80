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
    int64_t off;     // dense: offset (complex elements) of the [m][L][n] block;
                     // compressed: offset of its crank faces (m n each) in the face arena
    int32_t comp;    // 1: compressed along the frequencies (3D-ACA with dense faces)
    int32_t crank;   // compressed: number of crosses (0 for a zero block)
    int64_t foff;    // compressed: offset of its crank fibres (L each) in the fibre arena
};

// 3D-ACA of the near blocks with dense faces (csrc/near_aca.hip).
constexpr int kNearAcaMaxMN = 1024;     // larger blocks stay dense
constexpr int kNearAcaMaxFreq = 1024;
struct NearAcaOut {
    int32_t rank, capped, zero_faces, pad;
};
struct NearAcaArgs {
    const NearBlockDev *blocks;   // the problem's near blocks (dense offsets)
    int64_t b0;                   // first block of the chunk
    int32_t L, rc, mnmax, pad;    // frequencies, crosses per block slot, face slot size
    double eps, tie, delta;
    double2 *fib;                 // chunk scratch fibres [nblk][rc][L]
    NearAcaOut *out;              // [nblk]
};
void launch_near_aca(const NearAcaArgs &q, int nblk, const void *near, void *faces, int fp32,
                     hipStream_t st);
// dst: the operator's block table (comp, crank, off, foff set); face / fibre arenas of the
// compressed blocks, dense arena of the others
void launch_near_aca_pack(const NearAcaArgs &q, int nblk, const void *near, const void *faces,
                          const NearBlockDev *dst, void *face_arena, double2 *fib_arena,
                          void *dense_arena, int fp32, hipStream_t st);
void launch_near_aca_expand(const NearBlockDev &D, int L, const void *face_arena,
                            const double2 *fib_arena, double2 *out, int fp32, hipStream_t st);

// P1 double layer near field (every pair, all frequencies, FP64, stored as double2) and its
// entry test hook (far[p] != 0: 6-point rule on every triangle).
void launch_near_p1(const GeoDev &g, const QuadDev &q, const FreqDev &f, const NearPair *pairs,
                    int64_t npairs, const NearBlockDev *blocks, double2 *out64, hipStream_t st);
void launch_eval_p1(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                    const int32_t *rows, const int32_t *cols, const int32_t *ks,
                    const int32_t *far, double2 *out, hipStream_t st);

// Galerkin P1 operators (op 0 hypersingular, 1 adjoint double layer): near field and entry
// hook, as for the P1 double layer.
void launch_near_gp1(int op, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                     const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                     double2 *out64, hipStream_t st);
void launch_eval_gp1(int op, const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                     const int32_t *rows, const int32_t *cols, const int32_t *ks,
                     const int32_t *far, double2 *out, hipStream_t st);

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
// 1 collocation double layer, 2 Galerkin single layer; the face and tail launches also take
// -1, a joint build of both collocation operators (each block's kernel in FarBlockDev::kern).
//
// Far field 3D-ACA, run as iterations over all unfinished blocks of a batch; one iteration
// adds one face (one 3-D cross, or one zero face) to every active block in four phases:
//   face    residual face R = ENTRY(:, :, k) - sum_p coef_p H_p, all entries in parallel
//   aca     partial-pivot ACA of R, one workgroup per block (kinds 0-2: R and S in LDS, which
//           also expand H_l and pick the pivot; kind 3: R in HBM)
//   expand  kind 3: H_l = U W^T in 32 x 32 tiles with per-tile max, norm and Gram partials;
//           kinds 0-2: the Gram row of H_l (one partial row per face)
//   tail    pivot (kind 2), fibre, eq. (norm), stop test, next frequency and coefficients
constexpr int kFarChunk = 256;   // face entries per workgroup of the face phase
constexpr int kFarTile = 32;     // expand tile side
constexpr int kFarMaxRows = 8192; // rows / columns of a far block
__host__ __device__ constexpr int far_part_stride(int rcap) { return 2 + 2 * rcap; }

// One active block of an iteration (host-built, sorted kind 3, 2, 1, 0).
struct FarActive {
    int32_t b;          // batch-local block index
    int32_t ntile;      // expand tiles (kind 3)
    int64_t hslot;      // face-type element offset of this face's slot in the H pool
    int64_t fgslot;     // double2 offset of this cross's fibre (L) + Gram row (rcap) slot
    int64_t chunk0;     // first face-phase chunk
    int64_t tile0;      // first expand tile (kind 3) or the face's partial row (kinds 0-2)
};

struct FarCopy {        // one chunk of the factors of an accepted cross -> arena
    int32_t b, p, rho, chunk;
    int32_t which, pad;   // operator (arena) of a joint build
    int64_t off;
};
constexpr int kFarCopyChunk = 4096;   // elements per copy workgroup
struct FarGather {      // fibres of a finished block -> fibre arena
    int32_t b, rank;
    int32_t which, pad;   // operator (fibre arena) of a joint build
    int64_t off;
};

struct FarBatchDev {
    const FarBlockDev *blk;   // [nb]
    FarStateDev *st;          // [nb]
    double2 *coef;            // [nb][rcap] residual coefficients of the current face
    int64_t *hs, *fs;         // [nb][rcap] H slot / fibre slot of each accepted cross
    unsigned char *usedk;     // [nb][L]
    void *hpool;              // faces H_p (and the current residual), face type
    double2 *fgpool;          // fibres and Gram rows
    void *uw;                 // current face factors, face type
    double *part;             // expand partials, far_part_stride(rcap) doubles per tile
    int32_t *map_chunk;       // face chunk -> active index
    int32_t *map_tile;        // expand tile -> active index
    int32_t *status;          // [nact][2]: accepted | done << 1, rho
    FarMeta *meta;            // [nfar] (global index)
    CrossMeta *cmeta;         // [nfar][rcap]
    const double2 *dense;     // synthetic-entry mode: dense tensor [m][n][L] of block 0
    int32_t mixed, rcap, L, pad;
};

void launch_far_map(const FarBatchDev &bd, const FarActive *act, int nact, int nlarge,
                    hipStream_t st);
void launch_far_face(int kernel, const GeoDev &g, const FreqDev &f, const FarBatchDev &bd,
                     const FarActive *act, int64_t nchunk, hipStream_t st);
// Classes: kind 0 m n <= 1024, sides <= 64; kind 1 m n <= 2304, sides <= 96; kind 2 m n <=
// 4096 (FP64) or 8192 (mixed), sides <= 128; kind 3 larger.
// Kind 3 (R in HBM): threads 256, 512 or 1024; path 1: faces with m, n <= threads; 2: m, n
// <= kFarMultiE * 512 (512 threads); 0: any face.
constexpr int kFarMultiE = 5;
void launch_far_aca(int path, int threads, const AcaParams &P, const FarBatchDev &bd,
                    const FarActive *act, int nact, hipStream_t st);
// Kinds 0-2 (R and S in registers): faces with m n <= mnmax (576, 1024, 2304, or the kind-2
// bound) and workgroups of `threads` (64: one wave per face, 128, 256; kind 2: 512).
void launch_far_aca_small(int mnmax, int threads, const AcaParams &P, const FarBatchDev &bd,
                          const FarActive *act, int nact, hipStream_t st);
void launch_far_expand(const FarBatchDev &bd, const FarActive *act, int64_t ntile, hipStream_t st);
// Recompression of the current faces' factors (QR of both, SVD of the core, truncation at
// eps_aca), faces of rank 2..kRecMaxRank; nslot workgroups with kRecSlot doubles2 each of ws.
constexpr int kRecMaxRank = 128;
constexpr int64_t kRecSlot = 6 * (int64_t)kRecMaxRank * kRecMaxRank;
constexpr int kRecSlots = 256;   // concurrent faces (workgroups) of the recompression
void launch_far_recompress(const AcaParams &P, const FarBatchDev &bd, const FarActive *act,
                           int nact, double2 *ws, int nslot, hipStream_t st);
// Gram rows of LDS-resident faces (kinds 0-2) into their single partial row (FarActive::tile0)
void launch_far_gram_small(const FarBatchDev &bd, const FarActive *act, int nact, hipStream_t st);
void launch_far_tail(int kernel, const GeoDev &g, const FreqDev &f, const AcaParams &P,
                     const FarBatchDev &bd, const FarActive *act, int nact, int nlarge,
                     hipStream_t st);
// arena[w] / fib_arena[w]: output arenas of operator w (FarCopy::which, FarGather::which)
void launch_far_copy(const FarBatchDev &bd, const FarCopy *c, int n, void *const arena[2],
                     int64_t *cross_off, hipStream_t st);
void launch_far_gather(const FarBatchDev &bd, const FarGather *gt, int n, double2 *const fib_arena[2],
                       int64_t *fib_off, hipStream_t st);

// Test hook: entries of (row, col) tree positions with given tiers at frequency k.
// Mixed-precision far entries of one block (test hook): FP32 scaled entry times c_k in FP64.
void launch_eval_far_mixed(int kernel, const GeoDev &g, const FreqDev &f, const FarBlockDev &B,
                           int64_t n, const int32_t *il, const int32_t *jl, const int32_t *k,
                           double2 *out, hipStream_t st);
void launch_eval(int kernel, const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                 const int32_t *rows, const int32_t *cols, const int32_t *ks,
                 const int32_t *tiers, double2 *out, hipStream_t st);

// Apply (FP64, VALU reference path).
constexpr int kApplyCB = 8;   // most crosses per T = F X group of the VALU SUM apply
constexpr int kApplyKF = 64;  // fibre entries per LDS stage of that group
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
    int32_t nleaf, max_leaf_m;
    int32_t apply_cb;             // crosses per T group of the VALU SUM apply (1..kApplyCB)
    const int32_t *leaf_r0, *leaf_m;
    const int32_t *leaf_far_ptr, *leaf_far_idx;
    const int32_t *leaf_near_ptr, *leaf_near_idx;
    const int64_t *z_off;         // [nfar] offset of the block's z (sum_rho x nrhs) or v
    // near blocks compressed along the frequencies (NearBlockDev::comp): faces (near type,
    // [crank][m][n] at off), fibres ([crank][L] at foff), and for the SUM apply the vectors
    // T_l = sum_k f_l[k] X_k[tau] ([crank][n][nrhs] at tn_off[block])
    const void *near_faces;
    const double2 *near_fib;
    const int64_t *tn_off;
};
// Runge-Kutta gCQ history step (csrc/gcq.hip).
constexpr int kGcqMaxStages = 4;
struct GcqDev {
    int32_t L, m;                 // frequencies, stages
    int64_t M;                    // spatial unknowns
    double dt_prev, dt_cur;       // dt_{n-1}, dt_n
    double A[kGcqMaxStages * kGcqMaxStages];   // Butcher matrix, row-major m x m
    double g[kGcqMaxStages];      // b^T A^{-1}
    const double *w_re, *w_im;    // quadrature weights omega_l (device, L each)
};
void launch_gcq_history(const GcqDev &q, const double *s_re, const double *s_im,
                        const double2 *theta, double2 *x, double2 *W, hipStream_t st);

// Allocation-free apply: fixed per-device scratch array in apply.hip.
constexpr size_t kScratchBytes = 64ull << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;
// Takes the device address of the scratch array for `device` (which must be current) once;
// later calls return at once.
hipError_t scratch_setup(int device);
// The device address taken by scratch_setup, or nullptr before it.
void *scratch_address(int device);
// Workspace offsets of the VALU apply (z, t, per-block y) written on the device.
void launch_apply_offsets(const ApplyDev &a, int mode, int cb, int64_t *zoff, int64_t *toff,
                          int64_t *yoff, hipStream_t st);

// Matrix-core apply (SUM mode, complex64 right-hand sides), csrc/apply_mfma.hip.
constexpr int kMfmaMaxSumRho = 4096;   // sum of face ranks of one far block
constexpr int kMfmaMaxNearCols = 1024; // columns of one near block
constexpr int kMfmaMinRhs = 16;        // fewer right-hand sides take the VALU apply
// T = F X for the far blocks that share one column cluster tau: their fibre rows are
// stacked (rows of 32 per tile), so one slab X[:, tau, chunk] serves all of them.
struct MfmaTGroup {
    int32_t c0, n;        // column cluster (tree order)
    int32_t rows, m_tiles;
    int64_t row0;         // first row in the row table
};
struct MfmaTRow {         // one cross of one block
    int64_t f_off;        // its fibre (double2 offset in the fibre arena)
    int64_t t_off;        // its T row ([n][nrc], element offset)
};
struct MfmaZItem {        // Z_{b,l} rows [q0, q0 + 32)
    int32_t b, l, q0, pad;
    int64_t t_off, z_off; // T_b and Z_{b,l} offsets (elements)
};
struct MfmaApplyDev {
    int32_t nrc;          // columns of this chunk in T and Z (a power of two)
    int32_t lg_nrc;       // log2(nrc)
    int32_t ncur;         // right-hand sides of this chunk (<= nrc; the rest are zero)
    int32_t ldx, ldy;     // leading dimensions (nrhs) of X [L][M][nrhs] and Y [M][nrhs]
    int32_t c0;           // first right-hand side of the chunk
    const MfmaTGroup *t_groups;
    const int64_t *t_tile0;   // first tile of each group
    int32_t nt_groups;
    const MfmaTRow *t_rows;
    const MfmaZItem *z_items;
    const int64_t *z_off; // [nfar] Z_b offsets ([sum_rho][nrc])
    const int32_t *sum_rho;
};
void launch_apply_far_t(const ApplyDev &a, const MfmaApplyDev &d, int64_t ntiles, const float2 *X,
                        float2 *T, hipStream_t st);
void launch_apply_far_z(const ApplyDev &a, const MfmaApplyDev &d, int nitems, const float2 *T,
                        float2 *Z, hipStream_t st);
void launch_apply_leaf_mfma(const ApplyDev &a, const MfmaApplyDev &d, int row_tiles,
                            const float2 *X, const float2 *Z, float2 *Y, hipStream_t st);

// Side stream of the SUM apply: the far blocks run on it beside the near part (fork is
// recorded on the launch stream, join on the side stream; both created by the caller).
struct ApplySide {
    hipStream_t stream;
    hipEvent_t fork, join;
};

// x_fp32: X, Y and the workspace are complex64 (FP32 arithmetic), else complex128.
// Workspace pointers are in elements of that type.  side: null to launch everything on st.
void launch_apply(const ApplyDev &a, int mode, int x_fp32, const void *X, void *Y, void *Xp,
                  void *Yp, void *zbuf, void *tbuf, const int64_t *t_off, void *ybuf,
                  const int64_t *y_off, hipStream_t st, void *tnbuf = nullptr,
                  const ApplySide *side = nullptr);

}  // namespace gaca
