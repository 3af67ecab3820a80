// Reordered product eq. (product) of the compressed operator on the VALU:
//   SUM:      Y[:, b] = sum_l C(s_l) X_l[:, b]
//             far blocks: z_l = W_l^T (sum_k f_l[k] X_k[tau]),  y_b = sum_l U_l z_l
//             near blocks: Y[sigma] += sum_k N_k X_k[tau]
//   PER_FREQ: Y_k = C(s_k) X_k.
// Templated on the storage of factors / near field (FacT: double2 for the FP64 build,
// float2 for the mixed build) and on the right-hand sides (XT: complex128 or complex64),
// whose type also sets the arithmetic.  Owner-computes per leaf cluster: no atomics,
// every sum in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

template <class XT>
__global__ void permute_x_kernel(const XT *X, XT *Xp, const int64_t *perm, int L, int64_t M,
                                 int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)L * M * nrhs;
    if (t >= total) return;
    int c = (int)(t % nrhs);
    int64_t rest = t / nrhs;
    int64_t p = rest % M;
    int64_t l = rest / M;
    Xp[t] = X[(l * M + perm[p]) * nrhs + c];
}

template <class XT>
__global__ void scatter_y_kernel(const XT *Yp, XT *Y, const int64_t *perm, int nl, int64_t M,
                                 int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nl * M * nrhs;
    if (t >= total) return;
    int c = (int)(t % nrhs);
    int64_t rest = t / nrhs;
    int64_t p = rest % M;
    int64_t l = rest / M;
    Y[(l * M + perm[p]) * nrhs + c] = Yp[t];
}

// SUM: T = sum_k f_l[k] X_k[tau] (n x nrhs), z_l = W_l^T T for every cross of block b.
// PER_FREQ: v_l[q][k][c] = sum_j W_l[q][j] X_k[tau_j][c].
template <class FacT, class XT>
__global__ void __launch_bounds__(256) apply_far_a_kernel(ApplyDev a, int mode, const XT *Xp,
                                                          XT *zbuf, XT *tbuf, const int64_t *t_off) {
    const int b = blockIdx.x;
    const int m = a.far4[4 * b + 1], c0 = a.far4[4 * b + 2], n = a.far4[4 * b + 3];
    const FarMeta mt = a.meta[b];
    const int L = a.L, nr = a.nrhs;
    const int64_t M = a.M;
    XT *z = zbuf + a.z_off[b];
    XT *T = tbuf + t_off[b];
    const FacT *arena = reinterpret_cast<const FacT *>(a.arena);
    const double2 *F = a.fib_arena + a.fib_off[b];
    int64_t zo = 0;
    for (int c = 0; c < mt.rank; ++c) {
        const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + c];
        const FacT *W = arena + a.cross_off[(int64_t)b * a.rcap + c] + (int64_t)cm.rho * m;
        if (mode == 0) {
            for (int64_t t = threadIdx.x; t < (int64_t)n * nr; t += blockDim.x) {
                const int j = (int)(t / nr), cc = (int)(t - (int64_t)j * nr);
                XT acc = czero<XT>();
                for (int k = 0; k < L; ++k)
                    acc = cfma(cast_c<XT>(F[(int64_t)c * L + k]),
                               Xp[((int64_t)k * M + c0 + j) * nr + cc], acc);
                T[t] = acc;
            }
            __syncthreads();
            for (int64_t t = threadIdx.x; t < (int64_t)cm.rho * nr; t += blockDim.x) {
                const int qq = (int)(t / nr), cc = (int)(t - (int64_t)qq * nr);
                XT acc = czero<XT>();
                for (int j = 0; j < n; ++j)
                    acc = cfma(cast_c<XT>(W[(int64_t)qq * n + j]), T[(int64_t)j * nr + cc], acc);
                z[zo + t] = acc;
            }
            __syncthreads();
            zo += (int64_t)cm.rho * nr;
        } else {
            const int64_t cnt = (int64_t)cm.rho * L * nr;
            for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
                const int cc = (int)(t % nr);
                const int64_t rest = t / nr;
                const int k = (int)(rest % L);
                const int qq = (int)(rest / L);
                XT acc = czero<XT>();
                for (int j = 0; j < n; ++j)
                    acc = cfma(cast_c<XT>(W[(int64_t)qq * n + j]),
                               Xp[((int64_t)k * M + c0 + j) * nr + cc], acc);
                z[zo + t] = acc;
            }
            zo += cnt;
        }
    }
}

// SUM: y_b = sum_l U_l z_l for every far block (m x nrhs per block).
template <class FacT, class XT>
__global__ void __launch_bounds__(256) apply_far_y_kernel(ApplyDev a, const XT *zbuf, XT *ybuf,
                                                          const int64_t *y_off) {
    const int b = blockIdx.x;
    const int m = a.far4[4 * b + 1];
    const int nr = a.nrhs;
    const FarMeta mt = a.meta[b];
    const XT *z = zbuf + a.z_off[b];
    const FacT *arena = reinterpret_cast<const FacT *>(a.arena);
    for (int t = threadIdx.x; t < m * nr; t += blockDim.x) {
        const int r = t / nr, cc = t - r * nr;
        XT acc = czero<XT>();
        int64_t zo = 0;
        for (int c = 0; c < mt.rank; ++c) {
            const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + c];
            const FacT *U = arena + a.cross_off[(int64_t)b * a.rcap + c];
            for (int qq = 0; qq < cm.rho; ++qq)
                acc = cfma(cast_c<XT>(U[(int64_t)qq * m + r]), z[zo + (int64_t)qq * nr + cc], acc);
            zo += (int64_t)cm.rho * nr;
        }
        ybuf[y_off[b] + t] = acc;
    }
}

// SUM per leaf: Y[leaf rows] = sum over covering far blocks of y_b rows + near blocks'
// sum_k N_k X_k.  Outputs (row, rhs) are split over S thread groups that each take a
// share of the (near block, frequency) pairs; partial sums are added in a fixed order.
template <class NearT, class XT>
__global__ void __launch_bounds__(256) apply_leaf_sum_kernel(ApplyDev a, const XT *Xp,
                                                             const XT *ybuf, const int64_t *y_off,
                                                             XT *Yp) {
    __shared__ XT part[256];
    const int leaf = blockIdx.x;
    const int lr0 = a.leaf_r0[leaf], lm = a.leaf_m[leaf];
    const int L = a.L, nr = a.nrhs;
    const int64_t M = a.M;
    const int O = lm * nr;
    const int np0 = a.leaf_near_ptr[leaf], np1 = a.leaf_near_ptr[leaf + 1];
    const NearT *nearv = a.near64 ? reinterpret_cast<const NearT *>(a.near64)
                                  : reinterpret_cast<const NearT *>(a.near32);
    for (int o0 = 0; o0 < O; o0 += 256) {
        const int Oc = min(256, O - o0);
        const int S = max(1, 256 / Oc);
        const int t = threadIdx.x;
        const int s = t / Oc, o = o0 + (t - s * Oc);
        XT acc = czero<XT>();
        if (s < S) {
            const int r = o / nr, cc = o - r * nr;
            const int row = lr0 + r;
            const int npairs = (np1 - np0) * L;
            for (int e = s; e < npairs; e += S) {
                const NearBlockDev nb = a.nblocks[a.leaf_near_idx[np0 + e / L]];
                const int k = e - (e / L) * L;
                const int ro = row - nb.r0;
                const NearT *nrow = nearv + nb.off + ((int64_t)ro * L + k) * nb.n;
                const XT *xk = Xp + ((int64_t)k * M + nb.c0) * nr + cc;
                for (int j = 0; j < nb.n; ++j)
                    acc = cfma(cast_c<XT>(nrow[j]), xk[(int64_t)j * nr], acc);
            }
            if (s == 0) {
                for (int e = a.leaf_far_ptr[leaf]; e < a.leaf_far_ptr[leaf + 1]; ++e) {
                    const int b = a.leaf_far_idx[e];
                    const int ro = row - a.far4[4 * b];
                    acc = cadd(acc, ybuf[y_off[b] + (int64_t)ro * nr + cc]);
                }
            }
        }
        part[t] = acc;
        __syncthreads();
        if (t < Oc) {
            XT tot = part[t];
            for (int q = 1; q < S; ++q) tot = cadd(tot, part[q * Oc + t]);
            const int r = (o0 + t) / nr, cc = (o0 + t) - r * nr;
            Yp[(int64_t)(lr0 + r) * nr + cc] = tot;
        }
        __syncthreads();
    }
}

// PER_FREQ: one workgroup per (leaf, frequency); thread per (row, rhs).
template <class FacT, class NearT, class XT>
__global__ void __launch_bounds__(256) apply_leaf_freq_kernel(ApplyDev a, const XT *Xp,
                                                              const XT *zbuf, XT *Yp) {
    const int leaf = blockIdx.x;
    const int kf = blockIdx.y;
    const int lr0 = a.leaf_r0[leaf], lm = a.leaf_m[leaf];
    const int L = a.L, nr = a.nrhs;
    const int64_t M = a.M;
    const FacT *arena = reinterpret_cast<const FacT *>(a.arena);
    const NearT *nearv = a.near64 ? reinterpret_cast<const NearT *>(a.near64)
                                  : reinterpret_cast<const NearT *>(a.near32);
    for (int t = threadIdx.x; t < lm * nr; t += blockDim.x) {
        const int r = t / nr, cc = t - r * nr;
        const int row = lr0 + r;
        XT acc = czero<XT>();
        for (int e = a.leaf_far_ptr[leaf]; e < a.leaf_far_ptr[leaf + 1]; ++e) {
            const int b = a.leaf_far_idx[e];
            const int br0 = a.far4[4 * b], bm = a.far4[4 * b + 1];
            const int ro = row - br0;
            const FarMeta mt = a.meta[b];
            const XT *z = zbuf + a.z_off[b];
            const double2 *F = a.fib_arena + a.fib_off[b];
            int64_t zo = 0;
            for (int c = 0; c < mt.rank; ++c) {
                const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + c];
                const FacT *U = arena + a.cross_off[(int64_t)b * a.rcap + c];
                XT s = czero<XT>();
                for (int qq = 0; qq < cm.rho; ++qq)
                    s = cfma(cast_c<XT>(U[(int64_t)qq * bm + ro]),
                             z[zo + ((int64_t)qq * L + kf) * nr + cc], s);
                acc = cfma(cast_c<XT>(F[(int64_t)c * L + kf]), s, acc);
                zo += (int64_t)cm.rho * L * nr;
            }
        }
        for (int e = a.leaf_near_ptr[leaf]; e < a.leaf_near_ptr[leaf + 1]; ++e) {
            const NearBlockDev nb = a.nblocks[a.leaf_near_idx[e]];
            const int ro = row - nb.r0;
            const NearT *nrow = nearv + nb.off + ((int64_t)ro * L + kf) * nb.n;
            const XT *xk = Xp + ((int64_t)kf * M + nb.c0) * nr + cc;
            for (int j = 0; j < nb.n; ++j) acc = cfma(cast_c<XT>(nrow[j]), xk[(int64_t)j * nr], acc);
        }
        Yp[((int64_t)kf * M + row) * nr + cc] = acc;
    }
}

template <class FacT, class XT>
static void apply_impl(const ApplyDev &a, int mode, const XT *X, XT *Y, XT *Xp, XT *Yp, XT *zbuf,
                       XT *tbuf, const int64_t *t_off, XT *ybuf, const int64_t *y_off,
                       hipStream_t st) {
    const int64_t totx = (int64_t)a.L * a.M * a.nrhs;
    permute_x_kernel<XT><<<(unsigned)((totx + 255) / 256), 256, 0, st>>>(X, Xp, a.perm, a.L, a.M,
                                                                          a.nrhs);
    if (a.nfar > 0)
        apply_far_a_kernel<FacT, XT><<<a.nfar, 256, 0, st>>>(a, mode, Xp, zbuf, tbuf, t_off);
    const int nl = mode == 0 ? 1 : a.L;
    if (mode == 0) {
        if (a.nfar > 0) apply_far_y_kernel<FacT, XT><<<a.nfar, 256, 0, st>>>(a, zbuf, ybuf, y_off);
        apply_leaf_sum_kernel<FacT, XT><<<a.nleaf, 256, 0, st>>>(a, Xp, ybuf, y_off, Yp);
    } else {
        apply_leaf_freq_kernel<FacT, FacT, XT><<<dim3(a.nleaf, nl), 256, 0, st>>>(a, Xp, zbuf, Yp);
    }
    const int64_t toty = (int64_t)nl * a.M * a.nrhs;
    scatter_y_kernel<XT><<<(unsigned)((toty + 255) / 256), 256, 0, st>>>(Yp, Y, a.perm, nl, a.M,
                                                                         a.nrhs);
}

void launch_apply(const ApplyDev &a, int mode, int x_fp32, const void *X, void *Y, void *Xp,
                  void *Yp, void *zbuf, void *tbuf, const int64_t *t_off, void *ybuf,
                  const int64_t *y_off, hipStream_t st) {
#define GACA_APPLY(FT, XTT)                                                                  \
    apply_impl<FT, XTT>(a, mode, (const XTT *)X, (XTT *)Y, (XTT *)Xp, (XTT *)Yp, (XTT *)zbuf, \
                        (XTT *)tbuf, t_off, (XTT *)ybuf, y_off, st)
    if (a.fac_fp32) {
        if (x_fp32) GACA_APPLY(float2, float2);
        else GACA_APPLY(float2, double2);
    } else {
        if (x_fp32) GACA_APPLY(double2, float2);
        else GACA_APPLY(double2, double2);
    }
#undef GACA_APPLY
}

}  // namespace gaca
