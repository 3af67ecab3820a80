/*
 * gaca.h -- C ABI of the MI355X (gfx950) library for the generalised (3-D) adaptive cross
 * approximation of Laplace-domain boundary element tensors.
 *
 * Operation (Haider, Rjasanow, Schanz, "Generalised adaptive cross approximation for
 * convolution quadrature based boundary element formulation"):
 *   - Sec. 3 (spatial discretisation, eq. bie_semi_diri / bie_semi_indirect): the single
 *     layer V and double layer K matrices of flat triangles with piecewise-constant
 *     functions, collocation at element centroids or Galerkin;
 *   - Sec. 3 (temporal discretisation): their Laplace-domain kernels
 *     exp(-s r)/(4 pi r) and its normal derivative at the L complex frequencies s_l,
 *     i.e. the M x M x L array that the gCQ needs;
 *   - Sec. 4, Algorithm 1 and eq. (norm): 3D-ACA of every admissible block of a
 *     geometric cluster-tree partition (faces by ACA, pivot by dense expansion);
 *   - Sec. 4, eq. (product): the reordered product sum_l C(s_l) X_l.
 *
 * Conventions
 *   - every call returns a gaca_status; on failure gaca_last_error() (thread-local) holds
 *     a message; no C++ exception crosses the ABI;
 *   - complex numbers are interleaved (re, im) doubles (C128) or floats (C64);
 *   - element numbering is the caller's original order unless a function says "tree order"
 *     (the library renumbers elements so that every cluster is a contiguous range; the
 *     permutation is returned by gaca_problem_perm);
 *   - handles are owned by the library and freed by the matching *_destroy; all inputs are
 *     copied; a handle is used by one host thread at a time.  Destroying a context or a
 *     problem that still has problems or operators only marks it: it is freed with the last
 *     of them, so handles may be destroyed in any order.  Different problems of one
 *     context may be built from different threads at the same time (each problem has its
 *     own far-field streams and working memory), which overlaps their builds on the GPU.
 */
#ifndef GACA_H
#define GACA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GACA_ABI_VERSION 3

typedef enum {
    GACA_OK = 0,
    GACA_ERR_INVALID_ARG = -1,   /* bad argument (null pointer, size, degenerate mesh ...) */
    GACA_ERR_OOM = -2,           /* device allocation failed or exceeded max_device_bytes */
    GACA_ERR_HIP = -3,           /* a HIP runtime call failed */
    GACA_ERR_STATE = -4,         /* handle in the wrong state (e.g. no GPU, not built) */
    GACA_ERR_NOT_CONVERGED = -5, /* a rank cap was hit in at least one block (result kept) */
    GACA_ERR_UNSUPPORTED = -6    /* combination not implemented */
} gaca_status;

/* Discretisation (Sec. 3): collocation at the element centroids with piecewise constant
 * functions (single and double layer, eq. bie_semi_diri read with P0); Galerkin with
 * piecewise constant functions (single layer, eq. bie_semi_indirect); collocation at the
 * mesh vertices with piecewise linear continuous trial functions (double layer only,
 * eq. bie_semi_diri: K[i, j] = sum over the triangles around vertex j of the double layer
 * kernel at vertex i weighted by the hat function of j).  For GACA_COLLOCATION_P1 the
 * operator's rows and columns are the nv vertices (original vertex ids, tree-permuted like
 * the elements of the other schemes), precision must be GACA_FP64 and only GACA_DLP builds. */
/* GACA_GALERKIN_P1: the Galerkin operators of the Neumann problem (eq. bie_semi_neum) with
 * linear continuous test and trial functions, rows and columns the nv vertices as for
 * GACA_COLLOCATION_P1: the hypersingular operator GACA_HYP (in its form after integration by
 * parts: G_s times curl phi_i . curl phi_j plus s^2 n_x . n_y G_s phi_i phi_j) and the adjoint
 * double layer GACA_ADLP (dG/dn_x).  FP64 only.  Touching triangle pairs use the
 * Sauter-Schwab maps with n_touch Gauss points in each of the four variables. */
typedef enum {
    GACA_COLLOCATION_P0 = 0,
    GACA_GALERKIN_P0 = 1,
    GACA_COLLOCATION_P1 = 2,
    GACA_GALERKIN_P1 = 3
} gaca_scheme;
typedef enum { GACA_SLP = 0, GACA_DLP = 1, GACA_HYP = 2, GACA_ADLP = 3 } gaca_kernel;
/* FP64: every step in FP64.  MIXED: far-field faces evaluated and stored in FP32 complex
 * with a per-(block, frequency) scale, FP64 fibres, norms and pivot bookkeeping; near
 * field computed in FP64 and stored in FP32. */
typedef enum { GACA_FP64 = 0, GACA_MIXED = 1 } gaca_precision;
/* SUM: Y[i][b] = sum_l sum_j C(i,j,l) X[l][j][b]  (eq. product);
 * PER_FREQ: Y[l][i][b] = sum_j C(i,j,l) X[l][j][b]. */
typedef enum { GACA_APPLY_SUM = 0, GACA_APPLY_PER_FREQ = 1 } gaca_apply_mode;
typedef enum { GACA_C128 = 0, GACA_C64 = 1 } gaca_dtype;

typedef struct {
    int32_t leaf_size;        /* cluster-tree leaf size (default 32) */
    double eta;               /* admissibility: min(diam) <= eta * dist (default 1) */
    double eps3d;             /* 3-D ACA tolerance eps of Algorithm 1 (default 1e-6) */
    double eps_aca;           /* face ACA tolerance (default eps3d / 100) */
    gaca_precision precision; /* default GACA_FP64 */
    /* Quadrature orders (Sec. 3: Gauss rules chosen by a distance heuristic, Duffy for the
     * collocation singularity, regularising maps for the Galerkin singularities).  With
     * q = |x_i - x_j| / h the far blocks and near pairs with q >= 4 take the 6-point rule. */
    int32_t quad_mid;         /* collapsed Gauss points per direction, 2 <= q < 4 (default 4) */
    int32_t quad_near;        /* collocation: collapsed points per direction, q < 2 (default 8) */
    int32_t n_duffy;          /* Duffy order of the collocation self term (default 16) */
    int32_t n_galerkin;       /* Galerkin disjoint pairs with q < 2: outer and inner Duffy order
                                 per direction (default 5) */
    int32_t n_touch;          /* Galerkin pairs sharing an edge or a vertex: Gauss points per
                                 direction of the regularising maps (default 12) */
    double tie;               /* relative tie window of every argmax (default 1e-9, FP64) */
    double delta_zero;        /* zero-face threshold factor (default 1e-13) */
    int32_t max_rank3d;       /* cap on crosses per block (default min(L, 64)) */
    int32_t max_face_rank;    /* cap on a face's ACA rank (default min(m, n)) */
    uint64_t max_device_bytes;/* 0 = no limit; otherwise total library device memory cap */
    uint64_t batch_bytes;     /* far-field scratch per batch of blocks (default 160 GiB; at most
                                 half of the free device memory, or 60 % when all remaining
                                 blocks fit in one batch; the estimate takes the faces per block
                                 of the problem's last build of the operator); blocks enter the
                                 batches largest (m n) first; the result does not depend on the
                                 batches */
    int32_t threads_small;    /* face-ACA workgroup size for faces with m n <= 1024: 128
                                 (default) or 64 (one wave per face) */
    int32_t threads_large;    /* face-ACA workgroup size for the large faces (256, 512 or
                                 1024; default 0: chosen by the autotuner if autotune_cache is
                                 set, else 512) */
    int32_t verbose;          /* 1: one progress line per far-field batch on stderr */
    int32_t zero_rows_batch;  /* face ACA of the large faces, after a zero row: 1 (default)
                                 tries several unused rows per pass over the history, 0 one
                                 row per pass; both end at the same row */
    int32_t recompress;       /* 1: recompress every face after its ACA (QR of U and W, SVD of
                                 R_U R_W^T, truncation at eps_aca; Sec. 4 remarks), faces of
                                 rank 2..128; default 0 */
    int32_t pivot_estimate;   /* 0 (default): pivot of H_l by dense expansion; 1: eq. (index)
                                 estimate of the pivot row from the recompressed factors, the
                                 column from that row of H_l (needs recompress) */
    int32_t near_aca;         /* 1: after the build, compress each near block along the
                                 frequencies by 3D-ACA with dense faces (Sec. 4 remarks on the
                                 near field: rank r slices H_l (m x n, stored whole) times
                                 frequency fibres); a block stays dense where r (m n + L) >=
                                 m n L, where m n > 1024 or where the rank reaches
                                 min(L, 64).  Needs L <= 1024 (else GACA_ERR_UNSUPPORTED at
                                 problem creation).  The apply then runs on the VALU kernels
                                 (gaca_apply_noalloc: GACA_ERR_UNSUPPORTED).  Default 0 */
    const char *autotune_cache; /* NULL (default): no autotuning.  Otherwise a file path: the
                                 face-ACA workgroup sizes chosen for a workload (measured on
                                 the first build of a problem and timed per candidate) are
                                 read from and appended to this text file; the string is
                                 copied at problem creation */
} gaca_options;

typedef struct gaca_context gaca_context;
typedef struct gaca_problem gaca_problem;
typedef struct gaca_hmatrix gaca_hmatrix;

typedef struct {
    int64_t n_far, n_near;
    int32_t rank_min, rank_max;   /* 3-D ranks over far blocks (number of crosses) */
    double rank_mean;
    int32_t face_rank_max;
    double face_rank_mean;
    int64_t n_capped;             /* blocks that hit max_rank3d or max_face_rank */
    int64_t n_zero_blocks;        /* far blocks of rank 0 */
    uint64_t bytes_far;           /* stored far-field factors (U, W, fibres) */
    uint64_t bytes_near;          /* stored near field */
    double dense_bytes;           /* M * M * L * (16 FP64 / 8 MIXED) */
    double compression;           /* (bytes_far + bytes_near) / dense_bytes: stored bytes over
                                     the bytes of the dense tensor, the compression measure of
                                     Sec. 5.1 (cube example, compression figure) */
    double entries_near;          /* near-field tensor entries evaluated (m n L_eval per block:
                                     L_eval = ceil(L/2) when the frequencies are conjugate
                                     pairs, else L) */
    double entries_near_mirrored; /* near-field entries written as conjugates, not evaluated */
    double entries_face;          /* entries read by the face ACAs (algorithmic count) */
    double entries_fibre;         /* frequency-fibre entries (r L per block) */
    double entries_face_kernel;   /* entries the face kernels evaluated (dense faces) */
    double ms_near, ms_far, ms_total;  /* device time of the build phases */
    double ms_near_kernel;        /* sum of near-field kernel durations (HIP events) */
    double ms_far_kernel;         /* device time span of the far field (its iterations run
                                     on their own streams, concurrently with the near field) */
    int32_t n_far_launches;       /* far-field kernel launches */
    int32_t far_iters;            /* far-field iterations (faces of the longest block) */
    double far_flops;             /* algorithmic flops of the far field (FP64; faces in FP32
                                     arithmetic in the mixed path) */
    double far_kernel_evals;      /* quadrature-point x frequency kernel evaluations (far) */
    double near_kernel_evals;     /* quadrature-point x frequency kernel evaluations (near) */
    /* per far-field phase: 0 face (residual faces, every entry in parallel), 1 aca (face
     * ACA, one workgroup per block), 2 expand (dense H_l, pivot data and Gram values of
     * large faces), 3 tail (fibre, eq. (norm), stop test, next frequency) */
    double ms_far_phase[4];       /* sum of launch durations (HIP events on the launch stream) */
    int32_t launches_phase[4];
    double far_flops_phase[4];    /* algorithmic flops of the phase */
    double far_bytes_phase[4];    /* algorithmic HBM bytes of the phase: face = previous faces
                                     read once + the new face written (m n (l + 1) elements);
                                     expand = U, W read + H_l written + the previous faces read
                                     for the Gram row; aca and tail 0 (not modelled) */
    /* aca phase by launch class (device time of the class's launches on its stream): 0 m n <= 1024 and sides <= 64 (registers, 128 or 64 threads),
     * 1 m n <= 2304 and sides <= 96 (registers, 256 threads) together with the faces whose
     * sides are in (128, 256] when threads_large is above 256 (R in HBM, 256 threads, two
     * faces per CU), 2 m n <= 4096 and sides <= 128 (registers, 512 threads) together
     * with the larger faces whose sides are <= 128 (R in HBM, 256 threads), 3 the other
     * faces with a side above 128 (R in HBM, 512 threads by default) */
    double ms_far_by_kind[4];
    int32_t launches_by_kind[4];
    double far_flops_by_kind[4];  /* algorithmic flops of the class's face-ACA launches */
    /* class 3 by kernel path (far_aca_large_kernel instantiations): 0 general (sides above
     * the workgroup size, several entries per thread), 1 one row and one column entry per
     * thread (sides <= workgroup size), 2 several entries per thread (sides <= 5 x 512) */
    double ms_far_large_path[3];
    int32_t launches_large_path[3];
    double far_flops_large_path[3];
    int32_t threads_large_used;   /* workgroup size of the class-3 launches */
    int32_t threads_small_used;   /* workgroup size of the class-0 launches */
    int32_t autotune_state;       /* 0 sizes from the options, 1 chosen by timing each candidate
                                     during this problem's first build, 2 read from the
                                     autotune_cache file */
    double ms_far_aca_block_max;  /* longest total face-ACA time of one block (device clock) */
    double ms_host_setup;         /* host time of the build before the far-field launches */
    double ms_host_finish;        /* host time of the build after the far field completed */
    /* last matrix-core apply (SUM mode, complex64): device time, algorithmic flops (complex
     * multiply-add = 8), stored operator bytes it streamed (near field + factors + fibres) */
    double ms_apply;
    double apply_flops;
    double apply_operator_bytes;
    double ms_apply_part[3];      /* device time of the apply kernels: far T = F X, far Z = W T, leaf */
    double apply_flops_part[3];
    int32_t arena_in_place;       /* 1: the factor arena grows in place (virtual memory) */
    int32_t joint_build;          /* operators built together (gaca_build_both: 2); the far-field
                                     timings, launch counts, kernel evaluations and flops above
                                     then describe the shared launches of the joint build */
    /* near_aca: near blocks kept compressed, their mean and largest 3D-ACA rank, and the
     * host time of the compression pass (device work included) */
    int32_t near_rank_max;
    int64_t n_near_compressed;
    double near_rank_mean;
    double ms_near_aca;
} gaca_stats;

int gaca_abi_version(void);
const char *gaca_last_error(void);
void gaca_options_default(gaca_options *opt);

/* Context on HIP device `device`, launching on `hip_stream` (a hipStream_t, may be NULL
 * for the default stream; not owned).  GACA_ERR_STATE if no usable GPU.  Problems and
 * operators account their device memory in their context, and a destroyed problem hands its
 * far-field streams back to it for the next problem; the context is freed once it and all
 * of its problems are destroyed. */
gaca_status gaca_context_create(int device, void *hip_stream, gaca_context **out);
gaca_status gaca_context_destroy(gaca_context *ctx);
/* Device memory the library holds for this context (every problem and operator made on it,
 * and what they keep for reuse), in bytes.  Returns to 0 once every problem and operator of
 * the context is destroyed. */
gaca_status gaca_context_memory(const gaca_context *ctx, uint64_t *in_use);

/* Problem: mesh + frequencies + scheme (Sec. 3).  xyz: nv x 3 doubles; tri: M x 3 int32
 * vertex ids, counter-clockwise seen from outside; s_re, s_im: L frequencies.
 * Validates (finite coordinates, ids in range, non-degenerate triangles, L >= 1),
 * builds the cluster tree and block partition on the host and uploads the geometry.
 * If s_{L-1-l} == conj(s_l) exactly for all l, kernels evaluate only half the
 * frequencies and mirror the rest. */
gaca_status gaca_problem_create(gaca_context *ctx, const double *xyz, int64_t nv,
                                const int32_t *tri, int64_t M, const double *s_re,
                                const double *s_im, int32_t L, gaca_scheme scheme,
                                const gaca_options *opt, gaca_problem **out);
gaca_status gaca_problem_destroy(gaca_problem *p);
/* Tree permutation: perm[p] = original element id at tree position p (M entries). */
gaca_status gaca_problem_perm(const gaca_problem *p, int64_t *perm);
/* Block counts and lists (tree order): each block is (row_start, m, col_start, n). */
gaca_status gaca_problem_block_counts(const gaca_problem *p, int64_t *n_far, int64_t *n_near);
gaca_status gaca_problem_blocks(const gaca_problem *p, int64_t *far4, int64_t *near4);

/* Host-only tree + partition (no device), for tests of the host logic.
 * perm: M entries; far4 / near4: 4 * capacity entries; counts written to n_far, n_near;
 * GACA_ERR_INVALID_ARG if the capacity is too small (counts still written). */
gaca_status gaca_partition_host(const double *xyz, int64_t nv, const int32_t *tri, int64_t M,
                                int32_t leaf_size, double eta, int64_t *perm,
                                int64_t capacity, int64_t *far4, int64_t *n_far,
                                int64_t *near4, int64_t *n_near);
/* The same for the vertices of the P1 double layer (GACA_COLLOCATION_P1): split by vertex
 * position, admissibility (Sec. 4 remarks: purely geometric) on the boxes of the vertices'
 * patches (the triangles around each vertex, the supports of the hat functions).  perm: nv
 * entries.  GACA_ERR_INVALID_ARG also for a vertex that no triangle uses. */
gaca_status gaca_partition_host_p1(const double *xyz, int64_t nv, const int32_t *tri, int64_t M,
                                   int32_t leaf_size, double eta, int64_t *perm,
                                   int64_t capacity, int64_t *far4, int64_t *n_far,
                                   int64_t *near4, int64_t *n_near);

/* Host-only quadrature tables used by the kernels (Sec. 3 regular / Duffy quadrature):
 * kind 0: n-point Gauss-Legendre on [0, 1] -> nodes[n], weights[n];
 * kind 1: symmetric 6-point degree-4 triangle rule (n must be 6) -> nodes[6 * 3]
 *         barycentric coordinates, weights[6] summing to 1. */
gaca_status gaca_quadrature_rule(int kind, int n, double *nodes, double *weights);

/* Build (Algorithm 1 on every far block + dense near field) for one kernel.
 * Synchronous: returns when the device work is done.  GACA_ERR_NOT_CONVERGED if a rank
 * cap was hit (the handle is still returned and usable). */
gaca_status gaca_build(gaca_problem *p, gaca_kernel kernel, gaca_hmatrix **out);
/* Builds the single and double layer operators of a collocation problem together (Algorithm 1
 * on every far block of both; Sec. 4): the blocks of both operators advance in the same
 * far-field iterations, so each launch carries the faces of both; results are those of two
 * gaca_build calls.  GACA_ERR_UNSUPPORTED for a Galerkin problem.  GACA_ERR_NOT_CONVERGED as
 * gaca_build (both handles returned). */
gaca_status gaca_build_both(gaca_problem *p, gaca_hmatrix **slp_out, gaca_hmatrix **dlp_out);
/* An H-matrix refers to its problem: destroy it before the problem.  Destroying it waits
 * for the device to be idle; its factor and fibre arenas (when mapped in place and at most
 * an eighth of the device memory) are kept by the problem and reused by its next build,
 * and are freed with the problem. */
gaca_status gaca_hmatrix_destroy(gaca_hmatrix *h);
gaca_status gaca_hmatrix_stats(const gaca_hmatrix *h, gaca_stats *st);
/* Frequency-usage histogram: hist[k] = number of far blocks whose crosses use s_k (the
 * adaptively selected frequencies per block of Sec. 5.1, used-frequencies figure of the cube
 * example; with k_1 = 0 every block with a cross uses s_0).  hist: L entries (host). */
gaca_status gaca_hmatrix_freq_hist(const gaca_hmatrix *h, int64_t *hist);

/* Export of far block idx (tree-order rows/cols, see gaca_problem_blocks):
 * info[9] = {row_start, m, col_start, n, r, sum_rho, capped, zero_faces, aca_ticks}
 * (aca_ticks: device wall-clock ticks, 100 MHz, spent in the block's face ACAs).
 * Then (host buffers sized from info): ks[r], pi[r], pj[r] (tree-local pivots), rho[r],
 * U: sum_rho * m complex (cross by cross, column-major m x rho_l),
 * W: sum_rho * n complex (column-major n x rho_l), F: r * L complex (FP64 fibres),
 * all as C128 (MIXED factors are widened). */
gaca_status gaca_hmatrix_block_info(const gaca_hmatrix *h, int64_t idx, int64_t *info);
gaca_status gaca_hmatrix_block_export(const gaca_hmatrix *h, int64_t idx, int32_t *ks,
                                      int32_t *pi, int32_t *pj, int32_t *rho, double *U,
                                      double *W, double *F);
/* Near block idx as C128 [m][L][n] (tree-local order); a block compressed by near_aca is
 * expanded (sum over its slices H_l times fibre entries) on the device first. */
gaca_status gaca_hmatrix_near_export(const gaca_hmatrix *h, int64_t idx, double *out);
/* 3D-ACA rank of every near block (host int32[n_near], problem block order): the rank of a
 * block compressed by near_aca, -1 for a block stored dense (always -1 without near_aca). */
gaca_status gaca_hmatrix_near_ranks(const gaca_hmatrix *h, int32_t *ranks);

/* Apply (eq. product).  X: device pointer, [L][M][nrhs] complex in ORIGINAL element order;
 * Y: device pointer, [M][nrhs] (SUM) or [L][M][nrhs] (PER_FREQ).  dtype GACA_C128 runs the
 * FP64 apply, GACA_C64 the FP32 apply (SUM mode with nrhs >= 16: products on the matrix
 * cores, v_mfma_f32_16x16x4f32, FP32 sums).  Asynchronous on `hip_stream` (NULL: context
 * stream); X, Y are caller-owned; the library uses internal workspace sized at the
 * first call for this nrhs. */
gaca_status gaca_apply(gaca_hmatrix *h, gaca_apply_mode mode, int32_t nrhs, const void *X,
                       void *Y, gaca_dtype dtype, void *hip_stream);

/* Allocation-free apply, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * results as gaca_apply, computed with the VALU kernels of gaca_apply (no matrix-core path);
 * its workspace (tree-order copies of X and Y, the per-block z, T and y and their offsets)
 * lives in a fixed 64 MiB scratch array per device instead of memory allocated per operator.
 * The call allocates nothing and frees nothing.  GACA_ERR_INVALID_ARG if the workspace of
 * this operator, mode, nrhs and dtype exceeds 64 MiB (it grows as L M nrhs); GACA_ERR_STATE
 * if the operator's apply tables are missing.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (different streams or host threads) race and
 * must be serialised by the caller; the array keeps the last call's contents, and every byte
 * a call reads is written earlier in the same call. */
gaca_status gaca_apply_noalloc(gaca_hmatrix *h, gaca_apply_mode mode, int32_t nrhs, const void *X,
                               void *Y, gaca_dtype dtype, void *hip_stream);

/* Integration points s_l and weights omega_l of the generalised convolution quadrature
 * (App. A; Sec. 3, eq. (gcq_slp)) for a Runge-Kutta method with `stages` stages and Butcher
 * matrix rk_A (row-major stages x stages, nonsingular) and step sizes in [dt_min, dt_max]:
 * with lambda the eigenvalues of rk_A, q = dt_max max|lambda| / (dt_min min|lambda|) (times 5
 * for more than one stage, q > 1 required), k = (q - sqrt(2q-1)) / (q + sqrt(2q-1)),
 * h = dt_min min|lambda|, sigma_l = -K + (l + 1/2) 4K / n_q + i K'/2 (K = K(k^2),
 * K' = K(1 - k^2)), s_l = (sqrt(2q-1) (1/k + sn) / (1/k - sn) - 1) / (h (q - 1)) and
 * omega_l = 4K / (2 pi i n_q) gamma'(sigma_l) (Jacobi functions sn, cn, dn of parameter
 * k^2), so that sum_l omega_l F(s_l) is the quadrature of the Bromwich integral
 * (1 / 2 pi i) int F ds of eq. (conv_discrete).  The points are conjugate pairs,
 * s_{n_q-1-l} = conj(s_l) exactly (a problem made with them evaluates half of them).
 * Host only; outputs: n_q doubles each (host).  GACA_ERR_INVALID_ARG for q <= 1. */
gaca_status gaca_gcq_contour(int32_t stages, const double *rk_A, double dt_min, double dt_max,
                             int32_t n_q, double *s_re, double *s_im, double *w_re,
                             double *w_im);

/* History step of the Runge-Kutta gCQ (Sec. 3: eq. (gCQ_xn) and the sum of eq.
 * (gcq_formula)) with an operator built at the integration points (its problem's
 * frequencies s_l):
 *   x_{n-1}(s_l) = (I - dt_prev s_l A)^{-1} ((b^T A^{-1} x_{n-2}(s_l)) 1 + dt_prev A theta_{n-1}),
 *   W_l = omega_l (b^T A^{-1} x_{n-1}(s_l)) (I - dt_cur s_l A)^{-1} 1,
 *   Y = sum_l C(s_l) W_l   (gaca_apply, SUM mode, the stages as right-hand sides).
 * rk_A: stages x stages (row-major), rk_b: stages (host); w_re, w_im: the L weights (host).
 * Device buffers, complex128, original element order, caller-owned: theta_prev [M][stages]
 * (the stage values of step n-1), x [L][M][stages] (in: x_{n-2}, zero before the first
 * update; out: x_{n-1}), W [L][M][stages] (workspace, out: the vectors W_l), Y [M][stages]
 * (out: the history term).  Asynchronous on hip_stream as gaca_apply. */
gaca_status gaca_gcq_history(gaca_hmatrix *h, int32_t stages, const double *rk_A,
                             const double *rk_b, double dt_prev, double dt_cur,
                             const double *w_re, const double *w_im, const void *theta_prev,
                             void *x, void *W, void *Y, void *hip_stream);

/* Test hook: entries E(i[p], j[p], k[p]) (ORIGINAL element ids) with the quadrature the
 * build uses for a pair in a far block (far[p] = 1) or a near block (far[p] = 0), FP64,
 * evaluated on the device.  out: 2 * n doubles (host).  n may be 0. */
gaca_status gaca_eval_entries(gaca_problem *p, gaca_kernel kernel, int64_t n,
                              const int32_t *i, const int32_t *j, const int32_t *k,
                              const int32_t *far, double *out);

/* Test hook: entries of far block far_block (index into the far list of
 * gaca_problem_blocks) at tree-local rows il[p], columns jl[p] and frequency indices k[p], as
 * the mixed-precision face kernels evaluate them: FP32 arithmetic on the scaled kernel
 * exp(-s (r - d0)) / (4 pi r) (its normal derivative for the double layer; the Galerkin 6 x 6
 * rule for a Galerkin problem), where c_k = exp(-s_k d0) with d0 the distance of the block's
 * cluster box centres, then multiplied by c_k in FP64 (Sec. 3 kernels; the scaling is this
 * library's mixed-precision reading).  out: 2 n doubles (host).  n may be 0. */
gaca_status gaca_eval_far_entries_mixed(gaca_problem *p, gaca_kernel kernel, int64_t far_block,
                                        int64_t n, const int32_t *il, const int32_t *jl,
                                        const int32_t *k, double *out);

/* Test hook: 3D-ACA (Algorithm 1) of one dense tensor given on the device,
 * T[i][j][k] C128 with m x n x L entries, using the options' tolerances and precision
 * FP64.  The result has one far block covering the whole tensor. */
gaca_status gaca_compress_tensor(gaca_context *ctx, const void *dev_tensor, int64_t m,
                                 int64_t n, int32_t L, const gaca_options *opt,
                                 gaca_hmatrix **out);

#ifdef __cplusplus
}
#endif

#endif /* GACA_H */
