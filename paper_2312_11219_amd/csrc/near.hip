// Near-field kernels (dense over all frequencies) and the entry test hook.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "entries_dev.h"
#include "galerkin_dev.h"
#include "galerkin_p1_dev.h"
#include "kernels.h"

namespace gaca {

// Galerkin near field (single layer): one thread per (pair, NF frequencies), one class
// per launch.
template <int TIER, int NF>
__global__ void __launch_bounds__(256)
    near_gal_kernel(GeoDev g, QuadDev q, FreqDev f, const NearPair *__restrict__ pairs,
                    int64_t npairs, const NearBlockDev *__restrict__ blocks, double2 *out64,
                    float2 *out32) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const int l0 = blockIdx.y * NF;
    const int nl = min(NF, f.L_eval - l0);
    NearPair pr = pairs[p];
    NearBlockDev B = blocks[pr.blk];
    const int64_t i = B.r0 + pr.i, j = B.c0 + pr.j;
    double ar[NF], ai[NF];
    gal_near_entry<NF>(g, q, f, i, j, TIER, l0, nl, ar, ai);
    const int64_t base = B.off + (int64_t)pr.i * f.L * B.n + pr.j;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        if (t < nl) {
            const int l = l0 + t;
            if (out64) {
                out64[base + (int64_t)l * B.n] = make_double2(ar[t], ai[t]);
                if (f.mirror && f.L - 1 - l != l)
                    out64[base + (int64_t)(f.L - 1 - l) * B.n] = make_double2(ar[t], -ai[t]);
            } else {
                out32[base + (int64_t)l * B.n] = make_float2((float)ar[t], (float)ai[t]);
                if (f.mirror && f.L - 1 - l != l)
                    out32[base + (int64_t)(f.L - 1 - l) * B.n] =
                        make_float2((float)ar[t], (float)-ai[t]);
            }
        }
    }
}

template <int T, int NF>
static void near_gal_launch(const GeoDev &g, const QuadDev &q, const FreqDev &f,
                            const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                            double2 *o64, float2 *o32, hipStream_t st) {
    dim3 grid((unsigned)((npairs + 255) / 256), (unsigned)((f.L_eval + NF - 1) / NF));
    near_gal_kernel<T, NF><<<grid, 256, 0, st>>>(g, q, f, pairs, npairs, blocks, o64, o32);
}

void launch_near_galerkin(int tier, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                          const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                          double2 *out64, float2 *out32, hipStream_t st) {
    if (npairs <= 0) return;
    switch (tier) {
        case GT_FAR36: near_gal_launch<GT_FAR36, 8>(g, q, f, pairs, npairs, blocks, out64, out32, st); break;
        case GT_MID: near_gal_launch<GT_MID, 4>(g, q, f, pairs, npairs, blocks, out64, out32, st); break;
        case GT_NEAR: near_gal_launch<GT_NEAR, 2>(g, q, f, pairs, npairs, blocks, out64, out32, st); break;
        case GT_EDGE: near_gal_launch<GT_EDGE, 2>(g, q, f, pairs, npairs, blocks, out64, out32, st); break;
        case GT_VERTEX: near_gal_launch<GT_VERTEX, 2>(g, q, f, pairs, npairs, blocks, out64, out32, st); break;
        default: near_gal_launch<GT_COINC, 4>(g, q, f, pairs, npairs, blocks, out64, out32, st); break;
    }
}

__global__ void eval_gal_kernel(GeoDev g, QuadDev q, FreqDev f, int64_t n, const int32_t *rows,
                                const int32_t *cols, const int32_t *ks, const int32_t *tiers,
                                double2 *out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double ar[1], ai[1];
    gal_near_entry<1>(g, q, f, rows[p], cols[p], tiers[p], ks[p], 1, ar, ai);
    out[p] = make_double2(ar[0], ai[0]);
}

// One thread per (pair, chunk of NF frequencies) of one quadrature tier: every wave runs
// the same quadrature, so there is no divergence between tiers.  With mirrored
// frequencies only the first ceil(L/2) are evaluated; their conjugates fill the rest.
template <int KERNEL, int TIER, int NF>
__global__ void __launch_bounds__(256)
    near_kernel(GeoDev g, QuadDev q, FreqDev f, const NearPair *__restrict__ pairs,
                int64_t npairs, const NearBlockDev *__restrict__ blocks, double2 *out64,
                float2 *out32) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const int l0 = blockIdx.y * NF;
    const int nl = min(NF, f.L_eval - l0);
    NearPair pr = pairs[p];
    NearBlockDev B = blocks[pr.blk];
    const int64_t i = B.r0 + pr.i, j = B.c0 + pr.j;
    double ar[NF], ai[NF];
    near_entry<KERNEL, NF>(g, q, f, i, j, TIER, l0, nl, ar, ai);
    const int64_t base = B.off + (int64_t)pr.i * f.L * B.n + pr.j;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        if (t < nl) {
            const int l = l0 + t;
            if (out64) {
                out64[base + (int64_t)l * B.n] = make_double2(ar[t], ai[t]);
                if (f.mirror && f.L - 1 - l != l)
                    out64[base + (int64_t)(f.L - 1 - l) * B.n] = make_double2(ar[t], -ai[t]);
            } else {
                out32[base + (int64_t)l * B.n] = make_float2((float)ar[t], (float)ai[t]);
                if (f.mirror && f.L - 1 - l != l)
                    out32[base + (int64_t)(f.L - 1 - l) * B.n] =
                        make_float2((float)ar[t], (float)-ai[t]);
            }
        }
    }
}

template <int K, int T, int NF>
static void near_launch(const GeoDev &g, const QuadDev &q, const FreqDev &f,
                        const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                        double2 *o64, float2 *o32, hipStream_t st) {
    dim3 grid((unsigned)((npairs + 255) / 256), (unsigned)((f.L_eval + NF - 1) / NF));
    near_kernel<K, T, NF><<<grid, 256, 0, st>>>(g, q, f, pairs, npairs, blocks, o64, o32);
}

void launch_near(int kernel, int tier, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                 const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                 double2 *out64, float2 *out32, hipStream_t st) {
    if (npairs <= 0) return;
    // the expensive tiers (hundreds of points per pair) take one frequency per thread so
    // that there are enough threads; cheap tiers amortise the distance over 8 frequencies
#define GACA_NEAR(K, T, NF) near_launch<K, T, NF>(g, q, f, pairs, npairs, blocks, out64, out32, st)
    if (kernel == 0) {
        switch (tier) {
            case TIER_FAR6: GACA_NEAR(0, TIER_FAR6, 8); break;
            case TIER_MID4: GACA_NEAR(0, TIER_MID4, 8); break;
            case TIER_NEAR8: GACA_NEAR(0, TIER_NEAR8, 2); break;
            default: GACA_NEAR(0, TIER_SELF, 1); break;
        }
    } else {
        switch (tier) {
            case TIER_FAR6: GACA_NEAR(1, TIER_FAR6, 8); break;
            case TIER_MID4: GACA_NEAR(1, TIER_MID4, 8); break;
            case TIER_NEAR8: GACA_NEAR(1, TIER_NEAR8, 2); break;
            default: GACA_NEAR(1, TIER_SELF, 8); break;
        }
    }
#undef GACA_NEAR
}

// P1 double layer near field: one thread per (pair, NF frequencies); the quadrature tier
// is chosen per triangle of the column vertex's patch.
template <int NF>
__global__ void __launch_bounds__(256)
    near_p1_kernel(GeoDev g, QuadDev q, FreqDev f, const NearPair *__restrict__ pairs,
                   int64_t npairs, const NearBlockDev *__restrict__ blocks, double2 *out64) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const int l0 = blockIdx.y * NF;
    const int nl = min(NF, f.L_eval - l0);
    NearPair pr = pairs[p];
    NearBlockDev B = blocks[pr.blk];
    const int64_t i = B.r0 + pr.i, j = B.c0 + pr.j;
    double ar[NF], ai[NF];
    p1_entry<NF>(g, q, f, i, j, false, l0, nl, ar, ai);
    const int64_t base = B.off + (int64_t)pr.i * f.L * B.n + pr.j;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        if (t < nl) {
            const int l = l0 + t;
            out64[base + (int64_t)l * B.n] = make_double2(ar[t], ai[t]);
            if (f.mirror && f.L - 1 - l != l)
                out64[base + (int64_t)(f.L - 1 - l) * B.n] = make_double2(ar[t], -ai[t]);
        }
    }
}

void launch_near_p1(const GeoDev &g, const QuadDev &q, const FreqDev &f, const NearPair *pairs,
                    int64_t npairs, const NearBlockDev *blocks, double2 *out64, hipStream_t st) {
    if (npairs <= 0) return;
    constexpr int NF = 4;
    dim3 grid((unsigned)((npairs + 255) / 256), (unsigned)((f.L_eval + NF - 1) / NF));
    near_p1_kernel<NF><<<grid, 256, 0, st>>>(g, q, f, pairs, npairs, blocks, out64);
}

__global__ void eval_p1_kernel(GeoDev g, QuadDev q, FreqDev f, int64_t n, const int32_t *rows,
                               const int32_t *cols, const int32_t *ks, const int32_t *far,
                               double2 *out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double ar[1], ai[1];
    p1_entry<1>(g, q, f, rows[p], cols[p], far[p] != 0, ks[p], 1, ar, ai);
    out[p] = make_double2(ar[0], ai[0]);
}

void launch_eval_p1(const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                    const int32_t *rows, const int32_t *cols, const int32_t *ks,
                    const int32_t *far, double2 *out, hipStream_t st) {
    if (n <= 0) return;
    eval_p1_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(g, q, f, n, rows, cols, ks, far, out);
}

// Galerkin P1 operators of the Neumann problem (OP 0 hypersingular, 1 adjoint double layer):
// one thread per (pair, NF frequencies), every triangle pair of the two patches.
template <int OP, int NF>
__global__ void __launch_bounds__(256)
    near_gp1_kernel(GeoDev g, QuadDev q, FreqDev f, const NearPair *__restrict__ pairs,
                    int64_t npairs, const NearBlockDev *__restrict__ blocks, double2 *out64) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const int l0 = blockIdx.y * NF;
    const int nl = min(NF, f.L_eval - l0);
    NearPair pr = pairs[p];
    NearBlockDev B = blocks[pr.blk];
    const int64_t i = B.r0 + pr.i, j = B.c0 + pr.j;
    double ar[NF], ai[NF];
    gp1_entry<OP, NF>(g, q, f, i, j, false, l0, nl, ar, ai);
    const int64_t base = B.off + (int64_t)pr.i * f.L * B.n + pr.j;
#pragma unroll
    for (int t = 0; t < NF; ++t) {
        if (t < nl) {
            const int l = l0 + t;
            out64[base + (int64_t)l * B.n] = make_double2(ar[t], ai[t]);
            if (f.mirror && f.L - 1 - l != l)
                out64[base + (int64_t)(f.L - 1 - l) * B.n] = make_double2(ar[t], -ai[t]);
        }
    }
}

void launch_near_gp1(int op, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                     const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                     double2 *out64, hipStream_t st) {
    if (npairs <= 0) return;
    constexpr int NF = 2;
    dim3 grid((unsigned)((npairs + 255) / 256), (unsigned)((f.L_eval + NF - 1) / NF));
    if (op == 0) near_gp1_kernel<0, NF><<<grid, 256, 0, st>>>(g, q, f, pairs, npairs, blocks, out64);
    else near_gp1_kernel<1, NF><<<grid, 256, 0, st>>>(g, q, f, pairs, npairs, blocks, out64);
}

template <int OP>
__global__ void eval_gp1_kernel(GeoDev g, QuadDev q, FreqDev f, int64_t n, const int32_t *rows,
                                const int32_t *cols, const int32_t *ks, const int32_t *far,
                                double2 *out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double ar[1], ai[1];
    gp1_entry<OP, 1>(g, q, f, rows[p], cols[p], far[p] != 0, ks[p], 1, ar, ai);
    out[p] = make_double2(ar[0], ai[0]);
}

void launch_eval_gp1(int op, const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                     const int32_t *rows, const int32_t *cols, const int32_t *ks,
                     const int32_t *far, double2 *out, hipStream_t st) {
    if (n <= 0) return;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (op == 0) eval_gp1_kernel<0><<<nb, 256, 0, st>>>(g, q, f, n, rows, cols, ks, far, out);
    else eval_gp1_kernel<1><<<nb, 256, 0, st>>>(g, q, f, n, rows, cols, ks, far, out);
}

template <int KERNEL>
__global__ void eval_kernel(GeoDev g, QuadDev q, FreqDev f, int64_t n, const int32_t *rows,
                            const int32_t *cols, const int32_t *ks, const int32_t *tiers,
                            double2 *out) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double ar[1], ai[1];
    near_entry<KERNEL, 1>(g, q, f, rows[p], cols[p], tiers[p], ks[p], 1, ar, ai);
    out[p] = make_double2(ar[0], ai[0]);
}

void launch_eval(int kernel, const GeoDev &g, const QuadDev &q, const FreqDev &f, int64_t n,
                 const int32_t *rows, const int32_t *cols, const int32_t *ks,
                 const int32_t *tiers, double2 *out, hipStream_t st) {
    if (n <= 0) return;
    unsigned nb = (unsigned)((n + 127) / 128);
    if (kernel == 0)
        eval_kernel<0><<<nb, 128, 0, st>>>(g, q, f, n, rows, cols, ks, tiers, out);
    else if (kernel == 1)
        eval_kernel<1><<<nb, 128, 0, st>>>(g, q, f, n, rows, cols, ks, tiers, out);
    else
        eval_gal_kernel<<<nb, 128, 0, st>>>(g, q, f, n, rows, cols, ks, tiers, out);
}

}  // namespace gaca
