// Reordered product eq. (product) of the compressed operator, FP64 VALU path:
//   SUM:      Y[:, b] = sum_l C(s_l) X_l[:, b]
//             far blocks: z_l = W_l^T (sum_k f_l[k] X_k[tau]),  Y[sigma] += U_l z_l
//             near blocks: Y[sigma] += sum_k N_k X_k[tau]
//   PER_FREQ: Y_k = C(s_k) X_k.
// Owner-computes per leaf cluster (no atomics, deterministic).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

__global__ void permute_x_kernel(const double2 *X, double2 *Xp, const int64_t *perm, int L,
                                 int64_t M, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)L * M * nrhs;
    if (t >= total) return;
    int c = (int)(t % nrhs);
    int64_t rest = t / nrhs;
    int64_t p = rest % M;
    int64_t l = rest / M;
    Xp[t] = X[(l * M + perm[p]) * nrhs + c];
}

__global__ void scatter_y_kernel(const double2 *Yp, double2 *Y, const int64_t *perm, int nl,
                                 int64_t M, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nl * M * nrhs;
    if (t >= total) return;
    int c = (int)(t % nrhs);
    int64_t rest = t / nrhs;
    int64_t p = rest % M;
    int64_t l = rest / M;
    Y[(l * M + perm[p]) * nrhs + c] = Yp[t];
}

// SUM mode phase A: z_l = W_l^T (sum_k f_l[k] X_k[tau]) for every cross of block b.
// PER_FREQ phase A: v_l[q][k][c] = sum_j W_l[q][j] X_k[tau_j][c].
__global__ void __launch_bounds__(256) apply_far_a_kernel(ApplyDev a, int mode,
                                                          const double2 *Xp, double2 *zbuf,
                                                          double2 *tbuf, const int64_t *t_off) {
    const int b = blockIdx.x;
    const int r0 = a.far4[4 * b], m = a.far4[4 * b + 1], c0 = a.far4[4 * b + 2],
              n = a.far4[4 * b + 3];
    (void)r0;
    (void)m;
    const FarMeta mt = a.meta[b];
    const int L = a.L, nr = a.nrhs;
    const int64_t M = a.M;
    double2 *z = zbuf + a.z_off[b];
    double2 *T = tbuf + t_off[b];
    const double2 *F = a.fib_arena + a.fib_off[b];
    int64_t zo = 0;
    for (int c = 0; c < mt.rank; ++c) {
        const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + c];
        const double2 *W = a.arena + a.cross_off[(int64_t)b * a.rcap + c] + (int64_t)cm.rho * m;
        if (mode == 0) {
            for (int64_t t = threadIdx.x; t < (int64_t)n * nr; t += blockDim.x) {
                const int j = (int)(t / nr), cc = (int)(t - (int64_t)j * nr);
                double2 acc = make_double2(0.0, 0.0);
                for (int k = 0; k < L; ++k) {
                    double2 v = cmul(F[(int64_t)c * L + k], Xp[((int64_t)k * M + c0 + j) * nr + cc]);
                    acc.x += v.x;
                    acc.y += v.y;
                }
                T[t] = acc;
            }
            __syncthreads();
            for (int64_t t = threadIdx.x; t < (int64_t)cm.rho * nr; t += blockDim.x) {
                const int qq = (int)(t / nr), cc = (int)(t - (int64_t)qq * nr);
                double2 acc = make_double2(0.0, 0.0);
                for (int j = 0; j < n; ++j) {
                    double2 v = cmul(W[(int64_t)qq * n + j], T[(int64_t)j * nr + cc]);
                    acc.x += v.x;
                    acc.y += v.y;
                }
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
                double2 acc = make_double2(0.0, 0.0);
                for (int j = 0; j < n; ++j) {
                    double2 v = cmul(W[(int64_t)qq * n + j], Xp[((int64_t)k * M + c0 + j) * nr + cc]);
                    acc.x += v.x;
                    acc.y += v.y;
                }
                z[zo + t] = acc;
            }
            zo += cnt;
        }
    }
}

// Phase B: one workgroup per (leaf, frequency for PER_FREQ); thread per (row, rhs).
__global__ void __launch_bounds__(256) apply_leaf_kernel(ApplyDev a, int mode,
                                                         const double2 *Xp, const double2 *zbuf,
                                                         double2 *Yp) {
    const int leaf = blockIdx.x;
    const int kf = blockIdx.y;   // frequency (PER_FREQ) or 0
    const int lr0 = a.leaf_r0[leaf], lm = a.leaf_m[leaf];
    const int L = a.L, nr = a.nrhs;
    const int64_t M = a.M;
    for (int t = threadIdx.x; t < lm * nr; t += blockDim.x) {
        const int r = t / nr, cc = t - r * nr;
        const int row = lr0 + r;
        double2 acc = make_double2(0.0, 0.0);
        for (int e = a.leaf_far_ptr[leaf]; e < a.leaf_far_ptr[leaf + 1]; ++e) {
            const int b = a.leaf_far_idx[e];
            const int br0 = a.far4[4 * b], bm = a.far4[4 * b + 1];
            const int ro = row - br0;
            const FarMeta mt = a.meta[b];
            const double2 *z = zbuf + a.z_off[b];
            const double2 *F = a.fib_arena + a.fib_off[b];
            int64_t zo = 0;
            for (int c = 0; c < mt.rank; ++c) {
                const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + c];
                const double2 *U = a.arena + a.cross_off[(int64_t)b * a.rcap + c];
                if (mode == 0) {
                    for (int qq = 0; qq < cm.rho; ++qq) {
                        double2 v = cmul(U[(int64_t)qq * bm + ro], z[zo + (int64_t)qq * nr + cc]);
                        acc.x += v.x;
                        acc.y += v.y;
                    }
                    zo += (int64_t)cm.rho * nr;
                } else {
                    double2 s = make_double2(0.0, 0.0);
                    for (int qq = 0; qq < cm.rho; ++qq) {
                        double2 v = cmul(U[(int64_t)qq * bm + ro],
                                         z[zo + ((int64_t)qq * L + kf) * nr + cc]);
                        s.x += v.x;
                        s.y += v.y;
                    }
                    double2 v = cmul(F[(int64_t)c * L + kf], s);
                    acc.x += v.x;
                    acc.y += v.y;
                    zo += (int64_t)cm.rho * L * nr;
                }
            }
        }
        for (int e = a.leaf_near_ptr[leaf]; e < a.leaf_near_ptr[leaf + 1]; ++e) {
            const NearBlockDev nb = a.nblocks[a.leaf_near_idx[e]];
            const int ro = row - nb.r0;
            const int k0 = mode == 0 ? 0 : kf, k1 = mode == 0 ? L : kf + 1;
            for (int k = k0; k < k1; ++k) {
                const int64_t base = nb.off + ((int64_t)ro * L + k) * nb.n;
                for (int j = 0; j < nb.n; ++j) {
                    double2 nv;
                    if (a.near64) nv = a.near64[base + j];
                    else {
                        float2 t32 = a.near32[base + j];
                        nv = make_double2(t32.x, t32.y);
                    }
                    double2 v = cmul(nv, Xp[((int64_t)k * M + nb.c0 + j) * nr + cc]);
                    acc.x += v.x;
                    acc.y += v.y;
                }
            }
        }
        Yp[((int64_t)kf * M + row) * nr + cc] = acc;
    }
}

void launch_apply_fp64(const ApplyDev &a, int mode, const double2 *X, double2 *Y, double2 *Xp,
                       double2 *Yp, double2 *zbuf, double2 *tbuf, const int64_t *t_off,
                       hipStream_t st) {
    const int64_t totx = (int64_t)a.L * a.M * a.nrhs;
    permute_x_kernel<<<(unsigned)((totx + 255) / 256), 256, 0, st>>>(X, Xp, a.perm, a.L, a.M,
                                                                      a.nrhs);
    if (a.nfar > 0)
        apply_far_a_kernel<<<a.nfar, 256, 0, st>>>(a, mode, Xp, zbuf, tbuf, t_off);
    const int nl = mode == 0 ? 1 : a.L;
    apply_leaf_kernel<<<dim3(a.nleaf, nl), 256, 0, st>>>(a, mode, Xp, zbuf, Yp);
    const int64_t toty = (int64_t)nl * a.M * a.nrhs;
    scatter_y_kernel<<<(unsigned)((toty + 255) / 256), 256, 0, st>>>(Yp, Y, a.perm, nl, a.M,
                                                                     a.nrhs);
}

}  // namespace gaca
