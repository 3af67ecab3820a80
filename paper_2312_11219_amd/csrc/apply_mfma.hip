// Reordered product eq. (product), SUM mode, on the matrix cores: complex64 right-hand
// sides, FP32 products with FP32 accumulation (v_mfma_f32_16x16x4f32; a complex product is
// four real ones).  Factors and near field are read in their storage type (FP32 in the
// mixed build, FP64 otherwise) and rounded to FP32 as they are staged.
//
//   far blocks (tau = column cluster, r crosses):
//     T_b[l][j][c] = sum_k f_l[k] X_k[tau_j][c]           (r x L) . (L x n nrc)
//     Z_b[l][q][c] = sum_j W_l[q][j] T_b[l][j][c]          (rho_l x n) . (n x nrc)
//   per leaf (row tile of <= 32 rows, owner computes, no atomics):
//     Y[rows][c] = sum_near N[rows][(k, j)] X_k[tau_j][c] + sum_far U_b[rows][q] Z_b[q][c]
//
// Right-hand sides are processed in chunks of nrc columns; the permutation to tree order
// is applied by the loaders (X and Y stay in the caller's element order).  Sums are formed
// in segments of at most kFold K-elements (one block's contribution, or 256 terms) that are
// then added up, which keeps the FP32 accumulation error at the level of a 256-term sum.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kFold = 256;
constexpr int kSlicesPerStage = 1;   // K slices of 16 staged per barrier pair in kloop

__device__ __forceinline__ float2 to_f2(float2 v) { return v; }
__device__ __forceinline__ float2 to_f2(double2 v) { return make_float2((float)v.x, (float)v.y); }

// One 32 x TN complex tile of C += A B per workgroup of 256 threads (4 waves); wave w owns
// columns [w TN / 4, (w + 1) TN / 4) as 2 x TN/64 MFMA tiles of 16 x 16.  A and B are
// staged in LDS in slices of KS = 16 along K: As[k][r] (32 rows), Bs[k][c] (TN columns).
// Lane layout of the 16x16x4 instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 (l / 16) + t][l % 16], t = 0..3.
template <int TN>
struct CTile {
    static constexpr int KS = 16, TM = 32, WN = TN / 4, NJ = WN / 16;
    static_assert(NJ >= 1, "TN must be a multiple of 64");
    v4f cr[2][NJ], ci[2][NJ];
    __device__ void zero() {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) {
                cr[mi][nj] = v4f{0.f, 0.f, 0.f, 0.f};
                ci[mi][nj] = v4f{0.f, 0.f, 0.f, 0.f};
            }
    }
    __device__ void step(const float2 *As, const float2 *Bs) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int i = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + kq;
            float2 a[2], b[NJ];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) a[mi] = As[k * TM + 16 * mi + i];
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) b[nj] = Bs[k * TN + wave * WN + 16 * nj + i];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < NJ; ++nj) {
                    cr[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mi].x, b[nj].x, cr[mi][nj], 0, 0, 0);
                    cr[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[mi].y, b[nj].y, cr[mi][nj], 0, 0, 0);
                    ci[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mi].x, b[nj].y, ci[mi][nj], 0, 0, 0);
                    ci[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mi].y, b[nj].x, ci[mi][nj], 0, 0, 0);
                }
        }
    }
    // this += o, then o = 0 (two-level summation: segments of K are summed separately and
    // added up, so the FP32 rounding grows with the segment length, not with the whole K)
    __device__ void fold(CTile &o) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) {
                cr[mi][nj] += o.cr[mi][nj];
                ci[mi][nj] += o.ci[mi][nj];
                o.cr[mi][nj] = v4f{0.f, 0.f, 0.f, 0.f};
                o.ci[mi][nj] = v4f{0.f, 0.f, 0.f, 0.f};
            }
    }
    // visit every accumulated element: f(row, col, value), rows < 32, cols < TN
    template <class F>
    __device__ void visit(const F &f) const {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    f(16 * mi + 4 * (lane >> 4) + t, wave * WN + 16 * nj + (lane & 15),
                      make_float2(cr[mi][nj][t], ci[mi][nj][t]));
    }
};

// Stage A rows [0, 32) x K slice [k0, k0 + 16) into As[k][r]; a(r, k) returns the value,
// valid(r, k) whether it exists.  KMAJOR: consecutive threads walk k (row-major A), else r.
template <bool KMAJOR, class GA>
__device__ __forceinline__ void stage_a(float2 *As, int k0, int nrow, int kmax, const GA &ga) {
    for (int idx = threadIdx.x; idx < 16 * 32; idx += 256) {
        int r, k;
        if (KMAJOR) {
            r = idx >> 4;
            k = idx & 15;
        } else {
            k = idx >> 5;
            r = idx & 31;
        }
        const int kk = k0 + k;
        As[k * 32 + r] = (r < nrow && kk < kmax) ? ga(r, kk) : make_float2(0.f, 0.f);
    }
}

template <int TN, class GB>
__device__ __forceinline__ void stage_b(float2 *Bs, int k0, int kmax, int ncol, const GB &gb) {
    for (int idx = threadIdx.x; idx < 16 * TN; idx += 256) {
        const int k = idx / TN, c = idx - k * TN;
        const int kk = k0 + k;
        Bs[idx] = (kk < kmax && c < ncol) ? gb(kk, c) : make_float2(0.f, 0.f);
    }
}

// last index a with key[a] <= v (key ascending, key[0] = 0)
__device__ __forceinline__ int find_le(const int64_t *key, int n, int64_t v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (key[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One K loop of nslice slices of 16 on the matrix cores, software-pipelined: the operands of
// the next pair of slices are loaded into registers while the matrix cores work on the
// current pair (staged in LDS as As[k][32 rows], Bs[k][TN columns]).  pre(s) gives what
// slice s needs once per slice; ga(info, r, t) and gb(info, t, c) return its A and B
// elements (zero outside the operand).  KMAJOR_A: consecutive threads load consecutive t of
// one row (row-major A), else consecutive rows.  nk counts the K elements in seg since its
// last fold into acc; seg is folded once nk reaches kFold (the caller folds at the end of
// a block).
template <int TN, bool KMAJOR_A, class PRE, class GA, class GB>
__device__ __forceinline__ void kloop(CTile<TN> &acc, CTile<TN> &seg, int &nk, float2 *As, float2 *Bs,
                                      int nslice, const PRE &pre, const GA &ga, const GB &gb) {
    constexpr int PA = 16 * 32 / 256, PB = 16 * TN / 256, SP = kSlicesPerStage;
    const int tid = threadIdx.x;
    float2 ra[SP][PA], rb[SP][PB];
    auto load = [&](int s) {
#pragma unroll
        for (int h = 0; h < SP; ++h) {
            const int ss = s + h;
            const bool ok = ss < nslice;
            const auto info = pre(ok ? ss : 0);
#pragma unroll
            for (int i = 0; i < PA; ++i) {
                const int idx = tid + 256 * i;
                const int r = KMAJOR_A ? idx >> 4 : idx & 31, t = KMAJOR_A ? idx & 15 : idx >> 5;
                ra[h][i] = ok ? ga(info, r, t) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const int idx = tid + 256 * i;
                rb[h][i] = ok ? gb(info, idx / TN, idx % TN) : make_float2(0.f, 0.f);
            }
        }
    };
    load(0);
    for (int s = 0; s < nslice; s += SP) {
        if (nk >= kFold) {
            acc.fold(seg);
            nk = 0;
        }
        nk += 16 * SP;
        __syncthreads();
#pragma unroll
        for (int h = 0; h < SP; ++h) {
#pragma unroll
            for (int i = 0; i < PA; ++i) {
                const int idx = tid + 256 * i;
                const int r = KMAJOR_A ? idx >> 4 : idx & 31, t = KMAJOR_A ? idx & 15 : idx >> 5;
                As[h * 16 * 32 + t * 32 + r] = ra[h][i];
            }
#pragma unroll
            for (int i = 0; i < PB; ++i) Bs[h * 16 * TN + tid + 256 * i] = rb[h][i];
        }
        __syncthreads();
        if (s + SP < nslice) load(s + SP);
        seg.step(As, Bs);
        if (SP > 1 && s + 1 < nslice) seg.step(As + 16 * 32, Bs + 16 * TN);
    }
}

// ---------------------------------------------------------------------------------------
// T = F X for one column cluster: tile (group, row tile mt of the stacked crosses, column
// tile nt of (j, c)); the tiles of one column tile are consecutive, so the X slab they share
// stays in L2.
template <class FacT>
__global__ void __launch_bounds__(256)
    apply_far_t_kernel(ApplyDev a, MfmaApplyDev d, const float2 *X, float2 *T) {
    constexpr int TN = 256;
    __shared__ float2 As[kSlicesPerStage * 16 * 32];
    __shared__ float2 Bs[kSlicesPerStage * 16 * TN];
    __shared__ int sh_g;
    __shared__ int64_t fo[32], to[32];
    if (threadIdx.x == 0) sh_g = find_le(d.t_tile0, d.nt_groups, (int64_t)blockIdx.x);
    __syncthreads();
    const MfmaTGroup G = d.t_groups[sh_g];
    const int64_t tile = blockIdx.x - d.t_tile0[sh_g];
    const int mt = (int)(tile % G.m_tiles), nt = (int)(tile / G.m_tiles);
    const int L = a.L, nrc = d.nrc, n = G.n, c0b = G.c0;
    const int64_t ncols = (int64_t)n * nrc;
    const int r0 = 32 * mt, nrow = min(32, G.rows - r0);
    const int64_t n0 = (int64_t)nt * TN;
    if (threadIdx.x < nrow) {
        const MfmaTRow rw = d.t_rows[G.row0 + r0 + threadIdx.x];
        fo[threadIdx.x] = rw.f_off;
        to[threadIdx.x] = rw.t_off;
    }
    __syncthreads();
    CTile<TN> acc, seg;
    acc.zero();
    seg.zero();
    // with TN = 256 every B element a thread stages lies in its own column c = threadIdx.x:
    // the column's X offset is formed once
    const int64_t nn = n0 + threadIdx.x;
    const int jj = (int)(nn >> d.lg_nrc), cc = (int)(nn & (nrc - 1));
    const bool bok = nn < ncols && cc < d.ncur;
    const int64_t xoff = bok ? a.perm[c0b + jj] * (int64_t)d.ldx + d.c0 + cc : 0;
    const int64_t xk = a.M * (int64_t)d.ldx;
    int nk = 0;
    kloop<TN, true>(acc, seg, nk, As, Bs, (L + 15) >> 4,
        [&](int s) { return s << 4; },
        [&](int k0, int r, int t) {
            const int k = k0 + t;
            return (r < nrow && k < L) ? to_f2(a.fib_arena[fo[r] + k]) : make_float2(0.f, 0.f);
        },
        [&](int k0, int t, int) {
            const int k = k0 + t;
            return (k < L && bok) ? X[(int64_t)k * xk + xoff] : make_float2(0.f, 0.f);
        });
    acc.fold(seg);
    acc.visit([&](int r, int c, float2 v) {
        if (r < nrow && n0 + c < ncols) T[to[r] + n0 + c] = v;
    });
}

// Z_{b,l} = W_l T_l: tile (block b, cross l, row tile of rho_l, column tile).
template <class FacT>
__global__ void __launch_bounds__(256)
    apply_far_z_kernel(ApplyDev a, MfmaApplyDev d, const float2 *T, float2 *Z) {
    constexpr int TN = 64;
    __shared__ float2 As[kSlicesPerStage * 16 * 32];
    __shared__ float2 Bs[kSlicesPerStage * 16 * TN];
    const MfmaZItem it = d.z_items[blockIdx.x];
    const int b = it.b, l = it.l;
    const int n = a.far4[4 * b + 3], m = a.far4[4 * b + 1];
    const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + l];
    const FacT *W = reinterpret_cast<const FacT *>(a.arena) + a.cross_off[(int64_t)b * a.rcap + l] +
                    (int64_t)cm.rho * m;
    const int nrc = d.nrc;
    const int q0 = it.q0, c0 = blockIdx.y * TN;
    const float2 *Tl = T + it.t_off + (int64_t)l * n * nrc;
    CTile<TN> acc, seg;
    acc.zero();
    seg.zero();
    const int nrow = cm.rho - q0, ncl = nrc - c0;
    int nk = 0;
    kloop<TN, true>(acc, seg, nk, As, Bs, (n + 15) >> 4,
        [&](int s) { return s << 4; },
        [&](int k0, int r, int t) {
            const int k = k0 + t;
            return (r < nrow && k < n) ? to_f2(W[(int64_t)(q0 + r) * n + k]) : make_float2(0.f, 0.f);
        },
        [&](int k0, int t, int c) {
            const int k = k0 + t;
            return (k < n && c < ncl) ? Tl[(int64_t)k * nrc + c0 + c] : make_float2(0.f, 0.f);
        });
    acc.fold(seg);
    float2 *Zl = Z + it.z_off;
    acc.visit([&](int r, int c, float2 v) {
        if (q0 + r < cm.rho && c0 + c < nrc) Zl[(int64_t)(q0 + r) * nrc + c0 + c] = v;
    });
}

// Y rows of one leaf (row tile of 32) for one column tile: near blocks and far blocks of
// the leaf, one K stream per block.
template <class FacT, class NearT>
__global__ void __launch_bounds__(256)
    apply_leaf_mfma_kernel(ApplyDev a, MfmaApplyDev d, const float2 *X, const float2 *Z,
                           float2 *Y) {
    constexpr int TN = 64;
    __shared__ float2 As[kSlicesPerStage * 16 * 32];
    __shared__ float2 Bs[kSlicesPerStage * 16 * TN];
    __shared__ int64_t xrow[kMfmaMaxNearCols];
    const int leaf = blockIdx.x;
    const int lr0 = a.leaf_r0[leaf] + 32 * blockIdx.z, lm = min(32, a.leaf_m[leaf] - 32 * (int)blockIdx.z);
    if (lm <= 0) return;
    const int c0 = blockIdx.y * TN, nrc = d.nrc;
    const int L = a.L;
    const int64_t M = a.M;
    const NearT *nearv = a.near64 ? reinterpret_cast<const NearT *>(a.near64)
                                  : reinterpret_cast<const NearT *>(a.near32);
    const FacT *arena = reinterpret_cast<const FacT *>(a.arena);
    const int ncol = d.ncur - c0;
    CTile<TN> acc, seg;
    acc.zero();
    seg.zero();
    for (int e = a.leaf_near_ptr[leaf]; e < a.leaf_near_ptr[leaf + 1]; ++e) {
        const NearBlockDev nb = a.nblocks[a.leaf_near_idx[e]];
        const int ro = lr0 - nb.r0, n = nb.n;
        const int K = L * n, nj = (n + 15) >> 4;
        const NearT *A0 = nearv + nb.off + (int64_t)ro * K;
        const float2 *Xc = X + d.c0 + c0;
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += 256) xrow[j] = a.perm[nb.c0 + j] * (int64_t)d.ldx;
        __syncthreads();
        // slice s: frequency k = s / nj, columns j0 = 16 (s mod nj) + [0, 16)
        struct NearSlice {
            const NearT *a;      // A row 0 at column (k, j0)
            const float2 *x;     // X_k
            int j0;
        };
        int nk = 0;
        kloop<TN, true>(acc, seg, nk, As, Bs, L * nj,
            [&](int s) {
                const int k = s / nj, j0 = (s - k * nj) << 4;
                return NearSlice{A0 + (int64_t)k * n + j0, Xc + (int64_t)k * M * d.ldx, j0};
            },
            [&](const NearSlice &S, int r, int t) {
                return (r < lm && S.j0 + t < n) ? to_f2(S.a[(int64_t)r * K + t]) : make_float2(0.f, 0.f);
            },
            [&](const NearSlice &S, int t, int c) {
                return (S.j0 + t < n && c < ncol) ? S.x[xrow[S.j0 + t] + c] : make_float2(0.f, 0.f);
            });
        acc.fold(seg);
    }
    for (int e = a.leaf_far_ptr[leaf]; e < a.leaf_far_ptr[leaf + 1]; ++e) {
        const int b = a.leaf_far_idx[e];
        const int mb = a.far4[4 * b + 1], ro = lr0 - a.far4[4 * b];
        const int rank = a.meta[b].rank;
        const float2 *Zb = Z + d.z_off[b] + c0;
        int q0 = 0, nk = 0;
        for (int l = 0; l < rank && q0 < kMfmaMaxSumRho; ++l) {
            const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + l];
            const FacT *U = arena + a.cross_off[(int64_t)b * a.rcap + l] + ro;   // rho_l x mb
            const int rho = min(cm.rho, kMfmaMaxSumRho - q0);
            const float2 *Zl = Zb + (int64_t)q0 * nrc;
            kloop<TN, false>(acc, seg, nk, As, Bs, (rho + 15) >> 4,
                [&](int s) { return s << 4; },
                [&](int q0s, int r, int t) {
                    const int q = q0s + t;
                    return (r < lm && q < rho) ? to_f2(U[(int64_t)q * mb + r]) : make_float2(0.f, 0.f);
                },
                [&](int q0s, int t, int c) {
                    const int q = q0s + t;
                    return (q < rho && c0 + c < nrc) ? Zl[(int64_t)q * nrc + c] : make_float2(0.f, 0.f);
                });
            q0 += rho;
        }
        acc.fold(seg);
    }
    acc.visit([&](int r, int c, float2 v) {
        if (r < lm && c0 + c < d.ncur) Y[a.perm[lr0 + r] * d.ldy + d.c0 + c0 + c] = v;
    });
}

void launch_apply_far_t(const ApplyDev &a, const MfmaApplyDev &d, int64_t ntiles, const float2 *X,
                        float2 *T, hipStream_t st) {
    if (ntiles <= 0) return;
    if (a.fac_fp32) apply_far_t_kernel<float2><<<(unsigned)ntiles, 256, 0, st>>>(a, d, X, T);
    else apply_far_t_kernel<double2><<<(unsigned)ntiles, 256, 0, st>>>(a, d, X, T);
}

void launch_apply_far_z(const ApplyDev &a, const MfmaApplyDev &d, int nitems, const float2 *T,
                        float2 *Z, hipStream_t st) {
    if (nitems <= 0) return;
    dim3 grid(nitems, (d.nrc + 63) / 64);
    if (a.fac_fp32) apply_far_z_kernel<float2><<<grid, 256, 0, st>>>(a, d, T, Z);
    else apply_far_z_kernel<double2><<<grid, 256, 0, st>>>(a, d, T, Z);
}

void launch_apply_leaf_mfma(const ApplyDev &a, const MfmaApplyDev &d, int row_tiles,
                            const float2 *X, const float2 *Z, float2 *Y, hipStream_t st) {
    dim3 grid(a.nleaf, (d.nrc + 63) / 64, row_tiles);
    if (a.fac_fp32) apply_leaf_mfma_kernel<float2, float2><<<grid, 256, 0, st>>>(a, d, X, Z, Y);
    else apply_leaf_mfma_kernel<double2, double2><<<grid, 256, 0, st>>>(a, d, X, Z, Y);
}

}  // namespace gaca
