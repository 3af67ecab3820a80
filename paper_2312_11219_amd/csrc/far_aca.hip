// 3D-ACA of far (admissible) blocks: Algorithm 1 of the paper with ACA faces and the
// dense-expansion pivot, FP64 or mixed precision, run as iterations over all unfinished
// blocks of a batch.  One iteration adds one face to every active block:
//
//   face    R = ENTRY(:, :, k) - sum_{p < l} f_p[k] H_p         (previous dense faces H_p)
//   aca     partial-pivot ACA of R -> u_q, w_q; stop when |u||w| <= eps_aca sqrt(|C(:,:,k)|^2
//           + |S|^2), at a zero face, when all rows are used or at the face-rank cap
//   expand  H_l = sum_q u_q w_q^T (stored in the slot of R), max |H_l|^2, |H_l|_F^2 and the
//           Gram values <H_l, H_p>
//   tail    pivot (i_l, j_l) = tie-argmax |H_l|;
//           fibre f_l[k'] = (ENTRY(i_l, j_l, k') - sum_p H_p[i_l, j_l] f_p[k']) / H_l[i_l, j_l];
//           eq. (norm): |C^(l)|^2 += 2 Re sum_p <H_l, H_p><f_l, f_p> + |H_l|^2 |f_l|^2;
//           stop when |H_l| |f_l| <= eps |C^(l)|, else k_{l+1} = tie-argmax over unused k of
//           |f_l|; the residual coefficients and |C^(l)(:,:,k_{l+1})|^2 of the next face.
//
// The face phase evaluates every entry of every active face in parallel (the kernel
// evaluations are most of the arithmetic); only the ACA of one face is sequential and runs
// one workgroup per block.  Small faces (kinds 0/1) stay in LDS through the ACA, which
// updates R and S = sum_q u_q w_q^T in place and so also produces H_l = S, its pivot and its
// Gram row; larger faces keep R in HBM and are expanded by the tiled expand phase.
//
// Mixed precision: faces, residuals and face factors are FP32 (float2) and every face is
// kept divided by the block scale c_k = exp(-s_k d0) (d0 = distance of the cluster
// centres), so neither the e^{-Re(s) r} decay nor the phase Im(s) r leaves the FP32 range;
// the crosses stay exact because the scale moves into the FP64 fibres:
//   C ~ sum_p H~_p (x) f_p,  R~(:,:,k) = E(:,:,k)/c_k - sum_p (f_p[k]/c_k) H~_p.
// Fibres, Gram values, norms, stop tests and pivot comparisons are FP64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "entries_dev.h"
#include "galerkin_dev.h"
#include "galerkin_p1_dev.h"
#include "kernels.h"

namespace gaca {

constexpr int kMaxRowsLds = 8192;   // rows of a block (used-row flags in LDS)
constexpr int kMaxLds = 1024;       // frequencies
constexpr int kMaxRcap = 256;       // crosses per block
constexpr int kCoefLds = 512;       // staged history coefficients of the large-face ACA
constexpr int kCurRegs = 4;         // current u, w in registers for m, n <= 256
constexpr int kMultiE = kFarMultiE; // large faces: up to this many row / column entries per thread
constexpr int kBV = 1024;           // steps of a large face on the register paths (then the general one)

// Face entry at (il, jl, kk): FP64 value (FT = double2), the dense test tensor, or the
// scaled FP32 value (FT = float2).
template <int KERNEL, bool DENSE, class FT>
__device__ __forceinline__ FT face_entry(const GeoDev &g, const FreqDev &f, const double2 *dense,
                                         const FarBlockDev &B, int il, int jl, int kk) {
    if constexpr (KERNEL < 0) {   // joint build: the block's own collocation kernel
        return B.kern == 0 ? face_entry<0, DENSE, FT>(g, f, dense, B, il, jl, kk)
                           : face_entry<1, DENSE, FT>(g, f, dense, B, il, jl, kk);
    }
    if (DENSE) return from_d2<FT>(dense[((int64_t)il * B.n + jl) * f.L + kk]);
    const int64_t gi = B.r0 + il, gj = B.c0 + jl;
    if constexpr (KERNEL == 3) {   // P1 double layer (FP64 only)
        double er, ei;
        p1_far_entry(g, gi, gj, f.re[kk], f.im[kk], er, ei);
        return from_d2<FT>(make_double2(er, ei));
    } else if constexpr (KERNEL == 4 || KERNEL == 5) {   // Galerkin P1 D / K' (FP64 only)
        double er, ei;
        gp1_far_entry<KERNEL - 4>(g, QuadDev{}, gi, gj, f.re, f.im, kk, er, ei);
        return from_d2<FT>(make_double2(er, ei));
    } else if constexpr (KERNEL == 2) {
        if constexpr (sizeof(FT) == sizeof(double2)) {
            double er, ei;
            entry_gal36(g, gi, gj, f.re[kk], f.im[kk], er, ei);
            return from_d2<FT>(make_double2(er, ei));
        } else {
            const float cix = (float)(g.xx[gi] - B.xs_adj[0]), ciy = (float)(g.xy[gi] - B.xs_adj[1]),
                        ciz = (float)(g.xz[gi] - B.xs_adj[2]);
            const float cjx = (float)(g.xx[gj] - B.yt[0]), cjy = (float)(g.xy[gj] - B.yt[1]),
                        cjz = (float)(g.xz[gj] - B.yt[2]);
            return entry_gal36_scaled(g, cix, ciy, ciz, gi, B.Dh[0], B.Dh[1], B.Dh[2], B.d0f,
                                      B.kappa, gj, cjx, cjy, cjz, (float)f.re[kk], (float)f.im[kk]);
        }
    } else if constexpr (sizeof(FT) == sizeof(double2)) {
        double er, ei;
        entry_far6<KERNEL>(g, g.xx[gi], g.xy[gi], g.xz[gi], gj, f.re[kk], f.im[kk], er, ei);
        return from_d2<FT>(make_double2(er, ei));
    } else {
        const double xi = g.xx[gi], yi = g.xy[gi], zi = g.xz[gi];
        const float ax = (float)(xi - B.xs_adj[0]), ay = (float)(yi - B.xs_adj[1]),
                    az = (float)(zi - B.xs_adj[2]);
        const float cx = (float)(g.xx[gj] - B.yt[0]), cy = (float)(g.xy[gj] - B.yt[1]),
                    cz = (float)(g.xz[gj] - B.yt[2]);
        float num = 0.0f;
        if (KERNEL == 1) num = (float)(g.nx[gj] * xi + g.ny[gj] * yi + g.nz[gj] * zi - g.d[gj]);
        return entry_far6_scaled<KERNEL>(g, ax, ay, az, B.Dh[0], B.Dh[1], B.Dh[2], B.d0f,
                                         B.kappa, gj, cx, cy, cz, (float)f.re[kk],
                                         (float)f.im[kk], num);
    }
}

// Unscaled FP64 entry (fibres are always FP64).
template <int KERNEL, bool DENSE>
__device__ __forceinline__ double2 fibre_entry(const GeoDev &g, const FreqDev &f,
                                               const double2 *dense, const FarBlockDev &B,
                                               int il, int jl, int kk) {
    if constexpr (KERNEL < 0) {
        return B.kern == 0 ? fibre_entry<0, DENSE>(g, f, dense, B, il, jl, kk)
                           : fibre_entry<1, DENSE>(g, f, dense, B, il, jl, kk);
    }
    if (DENSE) return dense[((int64_t)il * B.n + jl) * f.L + kk];
    const int64_t gi = B.r0 + il, gj = B.c0 + jl;
    double er, ei;
    if constexpr (KERNEL == 3)
        p1_far_entry(g, gi, gj, f.re[kk], f.im[kk], er, ei);
    else if constexpr (KERNEL == 4 || KERNEL == 5)
        gp1_far_entry<KERNEL - 4>(g, QuadDev{}, gi, gj, f.re, f.im, kk, er, ei);
    else if constexpr (KERNEL == 2)
        entry_gal36(g, gi, gj, f.re[kk], f.im[kk], er, ei);
    else
        entry_far6<KERNEL>(g, g.xx[gi], g.xy[gi], g.xz[gi], gj, f.re[kk], f.im[kk], er, ei);
    return make_double2(er, ei);
}

// 1 / c_k = exp(s_k d0) (mixed scaling), FP64.
__device__ __forceinline__ double2 inv_scale(const FreqDev &f, const FarBlockDev &B, int k) {
    const double d0 = (double)B.d0f;
    const double mag = fm::exp(f.re[k] * d0);
    double sn, cs;
    fm::sincos(f.im[k] * d0, &sn, &cs);
    return make_double2(mag * cs, mag * sn);
}


template <bool MIXED>
using face_t = typename std::conditional<MIXED, float2, double2>::type;

// ---------------------------------------------------------------------------------------
// Work maps: face chunk -> active index, expand tile -> active index.
__global__ void far_map_kernel(FarBatchDev bd, const FarActive *act, int nact, int nlarge) {
    const int a = blockIdx.x;
    if (a >= nact) return;
    const FarActive A = act[a];
    const FarBlockDev B = bd.blk[A.b];
    const int64_t nch = ((int64_t)B.m * B.n + kFarChunk - 1) / kFarChunk;
    for (int64_t c = threadIdx.x; c < nch; c += blockDim.x) bd.map_chunk[A.chunk0 + c] = a;
    if (a < nlarge)
        for (int64_t t = threadIdx.x; t < A.ntile; t += blockDim.x) bd.map_tile[A.tile0 + t] = a;
}

// ---------------------------------------------------------------------------------------
// Face phase: R = ENTRY(:, :, k) - sum_p coef_p H_p into the face's H slot.
template <int KERNEL, bool DENSE, bool MIXED>
__global__ void __launch_bounds__(kFarChunk)
    far_face_kernel(GeoDev g, FreqDev f, FarBatchDev bd, const FarActive *act) {
    using FT = face_t<MIXED>;
    const int64_t c = blockIdx.x;
    const int a = bd.map_chunk[c];
    const FarActive A = act[a];
    const FarBlockDev B = bd.blk[A.b];
    const int ell = bd.st[A.b].ell, k = bd.st[A.b].k;
    __shared__ double2 coef[kMaxRcap];
    __shared__ int64_t hsl[kMaxRcap];
    for (int p = threadIdx.x; p < ell; p += kFarChunk) {
        coef[p] = bd.coef[(int64_t)A.b * bd.rcap + p];
        hsl[p] = bd.hs[(int64_t)A.b * bd.rcap + p];
    }
    __syncthreads();
    const int64_t mn = (int64_t)B.m * B.n;
    const int64_t idx = (c - A.chunk0) * kFarChunk + threadIdx.x;
    if (idx >= mn) return;
    const int i = (int)(idx / B.n), j = (int)(idx - (int64_t)i * B.n);
    const FT *H = reinterpret_cast<const FT *>(bd.hpool);
    FT e = face_entry<KERNEL, DENSE, FT>(g, f, bd.dense, B, i, j, k);
#pragma unroll 4
    for (int p = 0; p < ell; ++p) e = csub(e, cmul(from_d2<FT>(coef[p]), H[hsl[p] + idx]));
    reinterpret_cast<FT *>(bd.hpool)[A.hslot + idx] = e;
}

// ---------------------------------------------------------------------------------------
template <int NT, class T>
__device__ int tie_argmax_unused(const T *v, const unsigned char *used, int len, double tie2,
                                 Red<NT> &red) {
    double mx = -1.0;
    for (int t = threadIdx.x; t < len; t += NT)
        if (!used[t]) mx = fmax(mx, cabs2(v[t]));
    mx = red.max(mx);
    const double thr = tie2 * mx;
    int c = 0x7fffffff;
    for (int t = threadIdx.x; t < len; t += NT)
        if (!used[t] && cabs2(v[t]) >= thr) {
            c = t;
            break;
        }
    return red.imin(c);
}

template <int NT>
__device__ int first_unused(const unsigned char *used, int len, Red<NT> &red);

// As tie_argmax_unused, but never out of range: if no value compares (NaN), the first
// unused index (callers guarantee that one exists).
template <int NT, class T>
__device__ int pick_unused(const T *v, const unsigned char *used, int len, double tie2,
                           Red<NT> &red) {
    int c = tie_argmax_unused<NT>(v, used, len, tie2, red);
    if (c >= len) c = first_unused<NT>(used, len, red);
    return min(c, len - 1);
}

template <int NT>
__device__ int first_unused(const unsigned char *used, int len, Red<NT> &red) {
    int c = len;
    for (int t = threadIdx.x; t < len; t += NT)
        if (!used[t]) {
            c = t;
            break;
        }
    return red.imin(c);
}

// First row r >= r0 of the m x n face R (HBM) with an entry above zero_tol in modulus, or m;
// rows in chunks of about 16 NT entries.  A row is zero for the face ACA when the square
// root of its largest |R|^2 is at most zero_tol, i.e. when no entry exceeds it.
template <int NT, class FT>
__device__ int first_nonzero_row(const FT *R, int m, int n, int r0, double zero_tol, Red<NT> &red) {
    const int rb = max(1, 16 * NT / n);
    for (; r0 < m; r0 += rb) {
        const int r1 = min(m, r0 + rb);
        const int64_t cnt = (int64_t)(r1 - r0) * n;
        const FT *base = R + (int64_t)r0 * n;
        int c = m;
        for (int64_t idx = threadIdx.x; idx < cnt; idx += NT)
            if (sqrt(cabs2(base[idx])) > zero_tol) c = min(c, r0 + (int)(idx / n));
        c = red.imin(c);
        if (c < m) return c;
    }
    return m;
}

// Zero rows after the first cross.  A zero row sends the face ACA to the unused rows in
// index order until one has a residual entry above zero_tol; each try is a full pass over
// the history.  The large-face kernels try G rows per pass instead: the history is read once
// for all of them and every candidate's residual entries are formed by the same chain of
// operations as the row pass (terms of a padded step carry a zero coefficient and add an
// exact zero), so the first nonzero candidate is the row where the one-at-a-time search
// would stop; the zero ones before it are marked used.

// The G lowest unused rows from r0 up, ascending, in every lane of every wave (each wave
// scans for itself); returns their count (< G when fewer remain); c[g] past the count
// repeats the last row found.
template <int G>
__device__ int scan_unused(const unsigned char *used, int m, int r0, int (&c)[G]) {
    const int lane = threadIdx.x & 63;
    auto window = [&](int base) {
        const int r = base + lane;
        return (unsigned long long)__ballot(r < m && !used[r]);
    };
    unsigned long long bal = r0 < m ? window(r0) : 0ull;
    int cnt = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        while (bal == 0ull && r0 + 64 < m) {
            r0 += 64;
            bal = window(r0);
        }
        if (bal != 0ull) {
            c[g] = r0 + __ffsll(bal) - 1;
            bal &= bal - 1ull;
            cnt = g + 1;
        } else {
            c[g] = g > 0 ? c[g - 1] : 0;
        }
    }
    return cnt;
}

// Multi-entry layout (entries j = tid + NT e, e < NE): max_j |R(c_g, j) - sum_{q'<q}
// u_q'[c_g] w_q'[j]|^2 for each candidate, as one chain over q' per entry; the u
// coefficients of the HBM history are staged CH steps at a time in cs ([G][CH]), the w rows
// are loaded QZ steps at a time; wm holds NW * G doubles.  mx[g] is the same in every thread.
template <int NT, int G, int NE, int QZ, class FT>
__device__ void zero_rows_multi(const FT *R, const FT *Uh, const FT *Wh, const FT *Ub,
                                const FT *Wb, int m, int n, int q, int qL, const int (&c)[G],
                                FT *cs, int CH, double *wm, double (&mx)[G]) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int jj[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) jj[e] = min(tid + NT * e, n - 1);
    FT rv[G][NE], acc[G][NE];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            rv[g][e] = R[(int64_t)c[g] * n + jj[e]];
            acc[g][e] = czero<FT>();
        }
    const int qm = min(q, qL);
    for (int qq = 0; qq < qm; ++qq) {
        FT x[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) x[e] = Wh[qq * n + jj[e]];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const FT cg = Uh[qq * m + c[g]];
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[g][e] = cfma(cg, x[e], acc[g][e]);
        }
    }
    for (int qa = qL; qa < q; qa += CH) {
        const int nq = min(CH, q - qa);
        __syncthreads();
#pragma unroll
        for (int g = 0; g < G; ++g)
            for (int k = tid; k < nq; k += NT) cs[g * CH + k] = Ub[(int64_t)(qa + k) * m + c[g]];
        __syncthreads();
        for (int k = 0; k < nq; k += QZ) {
            FT x[QZ][NE];
#pragma unroll
            for (int qb = 0; qb < QZ; ++qb) {
                const FT *wp = Wb + (int64_t)(qa + min(k + qb, nq - 1)) * n;
#pragma unroll
                for (int e = 0; e < NE; ++e) x[qb][e] = wp[jj[e]];
            }
#pragma unroll
            for (int qb = 0; qb < QZ; ++qb) {
                const bool ok = k + qb < nq;
                const int kk = min(k + qb, nq - 1);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    FT cg = cs[g * CH + kk];
                    cg.x = ok ? cg.x : 0;
                    cg.y = ok ? cg.y : 0;
#pragma unroll
                    for (int e = 0; e < NE; ++e) acc[g][e] = cfma(cg, x[qb][e], acc[g][e]);
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double mv = 0.0;
#pragma unroll
        for (int e = 0; e < NE; ++e)
            if (tid + NT * e < n) mv = fmax(mv, cabs2(csub(rv[g][e], acc[g][e])));
        mv = wave_max(mv);
        if (lane == 0) wm[wave * G + g] = mv;
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double t = wm[g];
#pragma unroll
        for (int w = 1; w < NW; ++w) t = fmax(t, wm[w * G + g]);
        mx[g] = t;
    }
}

// One-entry layout with the history split over splitw thread groups (m, n <= NT): thread
// (s, j) sums steps [q s / splitw, q (s + 1) / splitw) in two interleaved accumulators,
// exactly as the row pass's history dot product does (LDS part in pairs, HBM part in groups
// of NB with the u coefficients from cs = [G][CL], q <= qL + CL; PF: the next
// group loaded during the arithmetic of this one); the group partials s >= 1 go through
// pp[g], and the row is R - p_0 - p_1 - ... as in the row pass.
template <int NT, int G, bool PF, int CL, class FT>
__device__ void zero_rows_split(const FT *R, const FT *Uh, const FT *Wh, const FT *Wb, int m,
                                int n, int q, int qL, int splitw, const int (&c)[G],
                                const FT *cs, FT *const (&pp)[G], double *wm, double (&mx)[G]) {
    constexpr int NW = NT / 64;
    constexpr int NB = NT >= 1024 ? 4 : 16;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    FT p[G], rv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        p[g] = czero<FT>();
        rv[g] = tid < n ? R[(int64_t)c[g] * n + tid] : czero<FT>();
    }
    if (tid < splitw * n) {
        const int s = tid / n, j = tid - s * n;
        const int q0 = (int)((int64_t)q * s / splitw), q1 = (int)((int64_t)q * (s + 1) / splitw);
        FT a0[G], a1[G];
#pragma unroll
        for (int g = 0; g < G; ++g) a0[g] = a1[g] = czero<FT>();
        const int qm = min(q1, qL);
        int qq = q0;
        for (; qq + 1 < qm; qq += 2) {
            const FT x0 = Wh[qq * n + j], x1 = Wh[(qq + 1) * n + j];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                a0[g] = cfma(Uh[qq * m + c[g]], x0, a0[g]);
                a1[g] = cfma(Uh[(qq + 1) * m + c[g]], x1, a1[g]);
            }
        }
        if (qq < qm) {
            const FT x0 = Wh[qq * n + j];
#pragma unroll
            for (int g = 0; g < G; ++g) a0[g] = cfma(Uh[qq * m + c[g]], x0, a0[g]);
        }
        qq = max(q0, qL);
        auto ld = [&](FT (&bv)[NB], int qs) {
#pragma unroll
            for (int t = 0; t < NB; ++t) bv[t] = Wb[(int64_t)(qs + t) * n + j];
        };
        auto fm = [&](const FT (&bv)[NB], int qs) {
#pragma unroll
            for (int t = 0; t < NB; t += 2)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    a0[g] = cfma(cs[g * CL + qs + t - qL], bv[t], a0[g]);
                    a1[g] = cfma(cs[g * CL + qs + t + 1 - qL], bv[t + 1], a1[g]);
                }
        };
        if constexpr (PF) {
            // the next group's loads in flight during this group's arithmetic
            const int ng = max(0, (q1 - qq) / NB);
            FT ba[NB], bb[NB];
            if (ng > 0) ld(ba, qq);
            for (int gi = 0; gi < ng; gi += 2) {
                if (gi + 1 < ng) ld(bb, qq + (gi + 1) * NB);
                fm(ba, qq + gi * NB);
                if (gi + 1 < ng) {
                    if (gi + 2 < ng) ld(ba, qq + (gi + 2) * NB);
                    fm(bb, qq + (gi + 1) * NB);
                }
            }
            qq += ng * NB;
        } else {
            for (; qq + NB <= q1; qq += NB) {
                FT bv[NB];
                ld(bv, qq);
                fm(bv, qq);
            }
        }
        for (; qq < q1; ++qq) {
            const FT x0 = Wb[(int64_t)qq * n + j];
#pragma unroll
            for (int g = 0; g < G; ++g) a0[g] = cfma(cs[g * CL + qq - qL], x0, a0[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            p[g] = cadd(a0[g], a1[g]);
            if (s > 0) pp[g][(s - 1) * n + j] = p[g];
        }
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double mv = 0.0;
        if (tid < n) {
            FT v = csub(rv[g], p[g]);
            for (int t = 1; t < splitw; ++t) v = csub(v, pp[g][(t - 1) * n + tid]);
            mv = cabs2(v);
        }
        mv = wave_max(mv);
        if (lane == 0) wm[wave * G + g] = mv;
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double t = wm[g];
#pragma unroll
        for (int w = 1; w < NW; ++w) t = fmax(t, wm[w * G + g]);
        mx[g] = t;
    }
}

// ---------------------------------------------------------------------------------------
// ACA phase, small faces: R and S = sum_q u_q w_q^T in registers, E = MNMAX / NT entries
// per thread (entry idx = tid + NT t), updated in place by the rank-1 steps; only the current
// row, column and w live in LDS, so several faces share a CU.  Also stores H_l = S over R and
// finds its max, norm and pivot (the Gram row against the previous faces follows in
// far_gram_small_kernel).
template <int NT, bool MIXED, int MNMAX, int SIDE>
__global__ void __launch_bounds__(NT, (NT == 256 && MNMAX == 2304) ? 3 : 1)
    far_aca_small_kernel(AcaParams P, FarBatchDev bd, const FarActive *act) {
    using FT = face_t<MIXED>;
    constexpr int E = MNMAX / NT;
    static_assert(E * NT == MNMAX, "MNMAX must be a multiple of NT");
    const FarActive A = act[blockIdx.x];
    const int b = A.b;
    const FarBlockDev B = bd.blk[b];
    const int m = B.m, n = B.n, mn = m * n;
    const int tid = threadIdx.x;
    const double zero_tol = bd.st[b].zero_tol, ref2 = bd.st[b].ref2;
    FT *R = reinterpret_cast<FT *>(bd.hpool) + A.hslot;
    FT *Ub = reinterpret_cast<FT *>(bd.uw) + B.uw_off;
    FT *Wb = Ub + (int64_t)B.rho_max * m;

    const int64_t t_start = wall_clock64();
    __shared__ FT rowv[SIDE];
    __shared__ FT ucol[SIDE];
    __shared__ FT wrow[SIDE];
    __shared__ unsigned char used_row[SIDE];
    __shared__ double redbuf[8 * (NT / 64) + 4];
    Red<NT> red{redbuf};
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);

    FT rr[E], ss[E];
    int ri[E];   // row of entry t; m for entries beyond the face
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = tid + NT * t;
        ri[t] = idx < mn ? idx / n : m;
        rr[t] = idx < mn ? R[idx] : czero<FT>();
        ss[t] = czero<FT>();
    }
    for (int r = tid; r < m; r += NT) used_row[r] = 0;
    int q = 0, i = 0, nused = 0;
    double s2 = 0.0;
    while (true) {
        // row i of the residual -> LDS (its owners write it)
#pragma unroll
        for (int t = 0; t < E; ++t)
            if (ri[t] == i) rowv[tid + NT * t - i * n] = rr[t];
        __syncthreads();
        double mx = 0.0;
        for (int j = tid; j < n; j += NT) mx = fmax(mx, cabs2(rowv[j]));
        mx = red.max(mx);
        if (tid == 0) used_row[i] = 1;
        ++nused;
        if (sqrt(mx) <= zero_tol) {
            // A zero row: the ACA goes on with the unused rows in index order, and every one
            // below the first with a nonzero residual entry is zero as well; find that row in
            // one pass over the register-held residual and mark the zero ones used.
            __syncthreads();
            int cand = m;
#pragma unroll
            for (int t = 0; t < E; ++t)
                if (ri[t] < m && !used_row[ri[t]] && sqrt(cabs2(rr[t])) > zero_tol) cand = min(cand, ri[t]);
            cand = red.imin(cand);
            double cnt = 0.0;
            for (int r = tid; r < cand; r += NT)
                if (!used_row[r]) cnt += 1.0;
            cnt = red.sum(cnt);
            for (int r = tid; r < cand; r += NT) used_row[r] = 1;
            nused += (int)cnt;
            if (cand >= m) break;
            i = cand;
            continue;
        }
        const double thr = tie2 * mx;
        int jc = n;
        for (int j = tid; j < n; j += NT)
            if (cabs2(rowv[j]) >= thr) {
                jc = j;
                break;
            }
        const int jp = min(red.imin(jc), n - 1);   // in range even for NaN rows
        const FT piv = rowv[jp];
        double nw2 = 0.0, nu2 = 0.0;
        for (int j = tid; j < n; j += NT) {
            const FT w = cdiv(rowv[j], piv);
            wrow[j] = w;
            Wb[(int64_t)q * n + j] = w;
            nw2 += cabs2(w);
        }
        // column jp of the residual (its owners write it)
#pragma unroll
        for (int t = 0; t < E; ++t)
            if (ri[t] < m && tid + NT * t - ri[t] * n == jp) {
                const FT u = rr[t];
                ucol[ri[t]] = u;
                Ub[(int64_t)q * m + ri[t]] = u;
                nu2 += cabs2(u);
            }
        __syncthreads();
        double sp = 0.0;
#pragma unroll
        for (int t = 0; t < E; ++t)
            if (ri[t] < m) {
                const FT tt = cmul(ucol[ri[t]], wrow[tid + NT * t - ri[t] * n]);
                rr[t] = csub(rr[t], tt);
                ss[t] = cadd(ss[t], tt);
                sp += cabs2(ss[t]);
            }
        // the maximum of |u_q|^2 over the unused rows (for the next-row pick) shares the
        // reduction round of the norms
        double mxu = -1.0;
        for (int r = tid; r < m; r += NT)
            if (!used_row[r]) mxu = fmax(mxu, cabs2(ucol[r]));
        red.sum3max(nu2, nw2, sp, mxu);
        s2 = sp;
        ++q;
        if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max)
            break;
        // next row: the lowest unused row with |u_q|^2 at the tie threshold of that maximum
        // (the first unused row if none compares)
        const double thu = tie2 * mxu;
        int c = 0x7fffffff;
        for (int r = tid; r < m; r += NT)
            if (!used_row[r] && cabs2(ucol[r]) >= thu) {
                c = r;
                break;
            }
        c = red.imin(c);
        if (c >= m) c = first_unused<NT>(used_row, m, red);
        i = min(c, m - 1);
    }
    const int rho = q;
    int pidx = 0;
    double mxh = 0.0, h2 = 0.0;
    if (rho > 0) {
#pragma unroll
        for (int t = 0; t < E; ++t)
            if (ri[t] < m) {
                R[tid + NT * t] = ss[t];
                const double a2 = cabs2(ss[t]);
                mxh = fmax(mxh, a2);
                h2 += a2;
            }
        red.maxsum(mxh, h2);
        const double thh = tie2 * mxh;
        int pc = 0x7fffffff;
#pragma unroll
        for (int t = E - 1; t >= 0; --t)   // lowest own index at the threshold
            if (ri[t] < m && cabs2(ss[t]) >= thh) pc = tid + NT * t;
        pidx = min(red.imin(pc), mn - 1);
    }
    if (tid == 0) {
        FarStateDev *S = bd.st + b;
        S->rho = rho;
        S->pidx = pidx;
        S->mxh = mxh;
        S->h2 = h2;
        S->aca_ticks += wall_clock64() - t_start;
    }
}

// ACA phase, large faces: R in HBM; the factor history u_q', w_q' in LDS for the first qL
// steps (as many as fit) and in HBM beyond, so the row / column corrections and the cross
// terms of the stopping norm mostly read LDS.  Row and column corrections are split over
// thread groups.
// PATH 1: faces with m, n <= NT (one entry per thread); 2: m, n <= kMultiE NT (several
// entries per thread, the general loop after kBV steps; NT = 512 only); 0: any face (general
// loop).  Each launch takes faces of one class, so each kernel holds only its own loops.
template <int NT, bool MIXED, int HB, int PATH>
__global__ void __launch_bounds__(NT)
    far_aca_large_kernel(AcaParams P, FarBatchDev bd, const FarActive *act) {
    using FT = face_t<MIXED>;
    const int64_t t_start = wall_clock64();
    const FarActive A = act[blockIdx.x];
    const int b = A.b;
    const FarBlockDev B = bd.blk[b];
    const int m = B.m, n = B.n;
    const int tid = threadIdx.x;
    constexpr int NW = NT / 64;
    const int wave = tid >> 6, lane = tid & 63;
    const double zero_tol = bd.st[b].zero_tol, ref2 = bd.st[b].ref2;
    const FT *R = reinterpret_cast<const FT *>(bd.hpool) + A.hslot;
    FT *Ub = reinterpret_cast<FT *>(bd.uw) + B.uw_off;
    FT *Wb = Ub + (int64_t)B.rho_max * m;

    __shared__ double2 hist_raw[HB / sizeof(double2)];
    __shared__ FT part[NT];       // split-K partial sums of row / column corrections
    // LDS sizes: the one-entry path (m, n <= NT, so at most NT rows and steps) needs used-row
    // flags and staged coefficients for NT rows / steps and Gram entries for NT steps (or the
    // zero-row candidates' coefficients, [G][CL]); the other paths the general bounds
    constexpr int CL = PATH == 1 && NT < kCoefLds ? NT : kCoefLds;
    constexpr int RL = PATH == 1 ? NT : kMaxRowsLds;
    constexpr int GZ = MIXED ? 4 : 2;
    constexpr int BZ = (int)(GZ * CL * sizeof(FT) / sizeof(double2));
    constexpr int BVL = PATH == 1 ? (NT > BZ ? NT : BZ) : kBV;
    __shared__ FT cbuf[CL];       // coefficients u_q'[i] / w_q'[jp] of the HBM part of the history
    __shared__ unsigned char used_row[RL];
    __shared__ double redbuf[8 * NW + 4];
    __shared__ double2 xbuf[NT];  // current w (face type), then split partials of v
    __shared__ double2 bvec[BVL];  // conj <w_q, w_q'> for q' < q
    Red<NT> red{redbuf};
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);
    const int qL = min(B.rho_max, (int)(HB / ((int64_t)(m + n) * (int64_t)sizeof(FT))));
    FT *Uh = reinterpret_cast<FT *>(hist_raw);       // [qL][m]
    FT *Wh = Uh + (int64_t)qL * m;                    // [qL][n]

    // sum_{q' in [q0, q1)} a_q'[ia] b_q'[ib] over the histories: the LDS part, then the HBM
    // part with the coefficients a_q'[ia] staged in cbuf (q' < qL + CL; sixteen loads
    // of b in flight), then any rest with both operands from HBM
    auto hdot = [&](const FT *ah, const FT *ag, int la, int ia, const FT *bh, const FT *bg,
                    int lb, int ib, int q0, int q1) {
        FT acc0 = czero<FT>(), acc1 = czero<FT>();
        const int qm = min(q1, qL);
        int qq = q0;
        for (; qq + 1 < qm; qq += 2) {
            acc0 = cfma(ah[qq * la + ia], bh[qq * lb + ib], acc0);
            acc1 = cfma(ah[(qq + 1) * la + ia], bh[(qq + 1) * lb + ib], acc1);
        }
        if (qq < qm) acc0 = cfma(ah[qq * la + ia], bh[qq * lb + ib], acc0);
        qq = max(q0, qL);
        const int qc = min(q1, qL + CL);
        constexpr int NB = NT >= 1024 ? 4 : 16;   // loads in flight (register budget)
        for (; qq + NB <= qc; qq += NB) {
            FT bv[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) bv[t] = bg[(int64_t)(qq + t) * lb + ib];
#pragma unroll
            for (int t = 0; t < NB; t += 2) {
                acc0 = cfma(cbuf[qq + t - qL], bv[t], acc0);
                acc1 = cfma(cbuf[qq + t + 1 - qL], bv[t + 1], acc1);
            }
        }
        for (; qq < qc; ++qq) acc0 = cfma(cbuf[qq - qL], bg[(int64_t)qq * lb + ib], acc0);
        FT acc = cadd(acc0, acc1);
        if (q1 > qc)
            acc = cadd(acc, dot_strided<FT, (NT >= 1024 ? 4 : 8)>(ag + ia, la, bg + ib, lb,
                                                                    max(q0, qc), q1));
        return acc;
    };
    // the same sum with both operands of the HBM part loaded per thread (the coefficient
    // a_q'[ia] is one address across the row, so no staging pass and barrier before it)
    // for every q' >= qL; used by the one-entry path
    auto hdot_direct = [&](const FT *ah, const FT *ag, int la, int ia, const FT *bh, const FT *bg,
                           int lb, int ib, int q0, int q1) {
        FT acc0 = czero<FT>(), acc1 = czero<FT>();
        const int qm = min(q1, qL);
        int qq = q0;
#pragma unroll 4
        for (; qq + 1 < qm; qq += 2) {
            acc0 = cfma(ah[qq * la + ia], bh[qq * lb + ib], acc0);
            acc1 = cfma(ah[(qq + 1) * la + ia], bh[(qq + 1) * lb + ib], acc1);
        }
        if (qq < qm) acc0 = cfma(ah[qq * la + ia], bh[qq * lb + ib], acc0);
        qq = max(q0, qL);
        constexpr int NB = NT >= 1024 ? 4 : 16;
        for (; qq + NB <= q1; qq += NB) {
            FT av[NB], bv[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                av[t] = ag[(int64_t)(qq + t) * la + ia];
                bv[t] = bg[(int64_t)(qq + t) * lb + ib];
            }
#pragma unroll
            for (int t = 0; t < NB; t += 2) {
                acc0 = cfma(av[t], bv[t], acc0);
                acc1 = cfma(av[t + 1], bv[t + 1], acc1);
            }
        }
        if (qq < q1) {
            // the rest (fewer than NB terms): its loads in flight together (indices clamped
            // into range), summed one at a time in order
            FT av[NB], bv[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const int qt = min(qq + t, q1 - 1);
                av[t] = ag[(int64_t)qt * la + ia];
                bv[t] = bg[(int64_t)qt * lb + ib];
            }
#pragma unroll
            for (int t = 0; t < NB; ++t)
                if (qq + t < q1) acc0 = cfma(av[t], bv[t], acc0);
        }
        return cadd(acc0, acc1);
    };
    // stage a_q'[ia] for q' in [qL, min(q, qL + CL)) (ends with a barrier)
    auto stage_coef = [&](const FT *ag, int la, int ia, int q) {
        const int nc = min(q, qL + CL) - qL;
        for (int t = tid; t < nc; t += NT) cbuf[t] = ag[(int64_t)(qL + t) * la + ia];
        __syncthreads();
    };

    for (int r = tid; r < m; r += NT) used_row[r] = 0;
    __syncthreads();
    int q = 0, i = 0, nused = 0;
    double s2 = 0.0;
    const int splitw = max(1, NT / n), splitu = max(1, NT / m);
    bool fin = false;   // the face ACA has ended (else the general path continues it)
    int fu = 0;   // every row below fu is used
    // the zero-row search after the first cross (see scan_unused): the row it ends at, or m
    auto zero_run = [&]() -> int {
        if constexpr (PATH == 2) {
            // candidates per pass: G NE accumulators per thread (register budget)
            auto pass = [&](auto gc, auto ec) -> int {
                constexpr int G = decltype(gc)::value, NE = decltype(ec)::value;
                constexpr int CH = (int)(BVL * sizeof(double2) / sizeof(FT)) / G;
                __syncthreads();
                int c[G];
                const int nc = scan_unused<G>(used_row, m, fu, c);
                if (nc == 0) return m;
                fu = c[0];
                double mx[G];
                zero_rows_multi<NT, G, NE, MIXED ? 8 : 4>(R, Uh, Wh, Ub, Wb, m, n, q, qL, c,
                                           reinterpret_cast<FT *>(bvec), CH,
                                           reinterpret_cast<double *>(xbuf), mx);
                int gs = nc;
#pragma unroll
                for (int g = G - 1; g >= 0; --g)
                    if (g < nc && !(sqrt(mx[g]) <= zero_tol)) gs = g;
                if (tid == 0)
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        if (g < gs) used_row[c[g]] = 1;
                nused += gs;
                if (gs < nc) {
                    int r = c[0];
#pragma unroll
                    for (int g = 1; g < G; ++g)
                        if (g == gs) r = c[g];
                    return r;
                }
                return nc < G ? m : -1;
            };
            using std::integral_constant;
            const int ne = min(kMultiE, (n + NT - 1) / NT);
            while (true) {
                int r;
                if (ne <= 1) r = pass(integral_constant<int, MIXED ? 8 : 4>{}, integral_constant<int, 1>{});
                else if (ne == 2) r = pass(integral_constant<int, MIXED ? 8 : 4>{}, integral_constant<int, 2>{});
                else if (ne == 3) r = pass(integral_constant<int, MIXED ? 6 : 3>{}, integral_constant<int, 3>{});
                else if (ne == 4) r = pass(integral_constant<int, MIXED ? 5 : 2>{}, integral_constant<int, 4>{});
                else r = pass(integral_constant<int, MIXED ? 4 : 2>{}, integral_constant<int, kMultiE>{});
                if (r >= 0) return r;
            }
        } else {
            constexpr int G = GZ;
            if (NT > CL || q > qL + CL) return first_unused<NT>(used_row, m, red);
            FT *cs = reinterpret_cast<FT *>(bvec);   // [G][CL]
            FT *pp[G];                               // [G][< NT] group partials
            if constexpr (MIXED) {
                pp[0] = part;
                pp[1] = cbuf;
                pp[2] = reinterpret_cast<FT *>(xbuf);
                pp[3] = pp[2] + NT;
            } else {
                pp[0] = part;
                pp[1] = reinterpret_cast<FT *>(xbuf);
            }
            while (true) {
                __syncthreads();
                int c[G];
                const int nc = scan_unused<G>(used_row, m, fu, c);
                if (nc == 0) return m;
                fu = c[0];
#pragma unroll
                for (int g = 0; g < G; ++g)
                    for (int k = tid; k < q - qL; k += NT) cs[g * CL + k] = Ub[(int64_t)(qL + k) * m + c[g]];
                __syncthreads();
                double mx[G];
                zero_rows_split<NT, G, MIXED, CL>(R, Uh, Wh, Wb, m, n, q, qL, splitw, c, cs, pp, redbuf, mx);
                int gs = nc;
#pragma unroll
                for (int g = G - 1; g >= 0; --g)
                    if (g < nc && !(sqrt(mx[g]) <= zero_tol)) gs = g;
                if (tid == 0)
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        if (g < gs) used_row[c[g]] = 1;
                nused += gs;
                if (gs < nc) {
                    int r = c[0];
#pragma unroll
                    for (int g = 1; g < G; ++g)
                        if (g == gs) r = c[g];
                    return r;
                }
                if (nc < G) return m;
            }
        }
    };
    if constexpr (PATH == 1) {
        fin = true;
        // One row entry and one column entry per thread, kept in registers.  The cross terms
        // sum_{q'<q} Re(<u_q, u_q'> <w_q, w_q'>) of the stopping norm are taken as
        // Re <u_q, v> with v = sum_{q'<q} conj(b_q') u_q', b_q' = <w_q, w_q'>: b is one
        // grouped pass over the w history, v is summed in the column pass, which reads the
        // u history anyway.
        FT *xw = reinterpret_cast<FT *>(xbuf);   // w_q (before the column pass)
        double2 *xv = xbuf;                      // split partials of v (column pass)
        while (true) {
            FT *Wq = Wb + (int64_t)q * n;
            FT *Uq = Ub + (int64_t)q * m;
            const FT rv = tid < n ? R[(int64_t)i * n + tid] : czero<FT>();
            if (tid < splitw * n) {
                const int s = tid / n, j = tid - s * n;
                const int q0 = (int)((int64_t)q * s / splitw), q1 = (int)((int64_t)q * (s + 1) / splitw);
                part[tid] = hdot_direct(Uh, Ub, m, i, Wh, Wb, n, j, q0, q1);
            }
            __syncthreads();
            FT v = rv;
            double mx = 0.0;
            if (tid < n) {
                for (int t = 0; t < splitw; ++t) v = csub(v, part[t * n + tid]);
                part[tid] = v;   // the only reader of part[tid] above is this thread
                mx = cabs2(v);
            }
            mx = red.max(mx);
            if (tid == 0) used_row[i] = 1;
            ++nused;
            if (sqrt(mx) <= zero_tol) {
                __syncthreads();
                int cand;
                if (q == 0) {
                    // no factors yet: the rows are visited in index order up to the first
                    // nonzero one, found in one pass over the face
                    cand = first_nonzero_row<NT>(R, m, n, i + 1, zero_tol, red);
                    for (int r = i + 1 + tid; r < cand; r += NT) used_row[r] = 1;
                    nused += cand - (i + 1);
                } else {
                    cand = P.zero_batch ? zero_run() : first_unused<NT>(used_row, m, red);
                }
                if (cand >= m) break;
                i = cand;
                continue;
            }
            const double thr = tie2 * mx;
            const int jp = min(red.imin(tid < n && cabs2(v) >= thr ? tid : n), n - 1);
            const FT piv = part[jp];
            const FT cv = tid < m ? R[(int64_t)tid * n + jp] : czero<FT>();
            double nw2 = 0.0;
            if (tid < n) {
                const FT w = cdiv(v, piv);
                Wq[tid] = w;
                if (q < qL) Wh[q * n + tid] = w;
                xw[tid] = w;
                nw2 = cabs2(w);
            }
            __syncthreads();
            if (q > 0) {
                // b_q' = <w_q, w_q'>: G lanes per q' (G a power of two, G q <= NT)
                int lg = 6;
                while (lg > 0 && (q << lg) > NT) --lg;
                const int G = 1 << lg, qq = tid >> lg, g = tid & (G - 1);
                double2 a0 = make_double2(0.0, 0.0), a1 = a0;
                if (qq < q) {
                    if (qq < qL) {
                        const FT *wp = Wh + qq * n;
#pragma unroll 4
                        for (int j = g; j < n; j += G) a0 = cfma(to_d2(xw[j]), conj_d2(to_d2(wp[j])), a0);
                    } else {
                        const FT *wp = Wb + (int64_t)qq * n;
                        constexpr int NBW = 8;
                        int j = g;
                        for (; j + (NBW - 1) * G < n; j += NBW * G) {
                            FT wv[NBW];
#pragma unroll
                            for (int t = 0; t < NBW; ++t) wv[t] = wp[j + t * G];
#pragma unroll
                            for (int t = 0; t < NBW; t += 2) {
                                a0 = cfma(to_d2(xw[j + t * G]), conj_d2(to_d2(wv[t])), a0);
                                a1 = cfma(to_d2(xw[j + (t + 1) * G]), conj_d2(to_d2(wv[t + 1])), a1);
                            }
                        }
                        if (j < n) {
                            // the rest in one round of loads (indices clamped into range),
                            // summed in order
                            FT wv[NBW];
#pragma unroll
                            for (int t = 0; t < NBW; ++t) wv[t] = wp[min(j + t * G, n - 1)];
#pragma unroll
                            for (int t = 0; t < NBW; ++t)
                                if (j + t * G < n) a0 = cfma(to_d2(xw[min(j + t * G, n - 1)]), conj_d2(to_d2(wv[t])), a0);
                        }
                    }
                }
                a0 = cadd(a0, a1);
                for (int o = G >> 1; o > 0; o >>= 1) {
                    a0.x += __shfl_xor(a0.x, o, 64);
                    a0.y += __shfl_xor(a0.y, o, 64);
                }
                if (g == 0 && qq < q) bvec[qq] = conj_d2(a0);
                __syncthreads();
            }
            if (tid < splitu * m) {
                // column jp of R - sum_{q'<q} w_q'[jp] u_q', and v, over this thread's q' (the
                // coefficients w_q'[jp] of the HBM part loaded per thread, one address per row)
                const int s = tid / m, r = tid - s * m;
                const int q0 = (int)((int64_t)q * s / splitu), q1 = (int)((int64_t)q * (s + 1) / splitu);
                FT c0 = czero<FT>(), c1 = czero<FT>();
                double2 v0 = make_double2(0.0, 0.0), v1 = v0;
                const int qm = min(q1, qL);
                int qq = q0;
#pragma unroll 4
                for (; qq < qm; ++qq) {
                    const FT uu = Uh[qq * m + r];
                    c0 = cfma(Wh[qq * n + jp], uu, c0);
                    v0 = cfma(bvec[qq], to_d2(uu), v0);
                }
                qq = max(q0, qL);
                constexpr int NB = NT >= 1024 ? 4 : 16;
                for (; qq + NB <= q1; qq += NB) {
                    FT uv[NB], wv[NB];
#pragma unroll
                    for (int t = 0; t < NB; ++t) {
                        uv[t] = Ub[(int64_t)(qq + t) * m + r];
                        wv[t] = Wb[(int64_t)(qq + t) * n + jp];
                    }
#pragma unroll
                    for (int t = 0; t < NB; t += 2) {
                        c0 = cfma(wv[t], uv[t], c0);
                        c1 = cfma(wv[t + 1], uv[t + 1], c1);
                        v0 = cfma(bvec[qq + t], to_d2(uv[t]), v0);
                        v1 = cfma(bvec[qq + t + 1], to_d2(uv[t + 1]), v1);
                    }
                }
                if (qq < q1) {
                    // the rest in one round of loads (clamped), summed in order
                    FT uv[NB], wv[NB];
#pragma unroll
                    for (int t = 0; t < NB; ++t) {
                        const int qt = min(qq + t, q1 - 1);
                        uv[t] = Ub[(int64_t)qt * m + r];
                        wv[t] = Wb[(int64_t)qt * n + jp];
                    }
#pragma unroll
                    for (int t = 0; t < NB; ++t)
                        if (qq + t < q1) {
                            c0 = cfma(wv[t], uv[t], c0);
                            v0 = cfma(bvec[min(qq + t, q1 - 1)], to_d2(uv[t]), v0);
                        }
                }
                part[tid] = cadd(c0, c1);
                xv[tid] = cadd(v0, v1);
            }
            __syncthreads();
            double nu2 = 0.0, cr = 0.0, mxu = -1.0;
            FT u = cv;
            if (tid < m) {
                double2 vs = make_double2(0.0, 0.0);
                for (int t = 0; t < splitu; ++t) {
                    u = csub(u, part[t * m + tid]);
                    vs = cadd(vs, xv[t * m + tid]);
                }
                Uq[tid] = u;
                if (q < qL) Uh[q * m + tid] = u;
                nu2 = cabs2(u);
                const double2 ud = to_d2(u);
                cr = ud.x * vs.x + ud.y * vs.y;
                if (!used_row[tid]) mxu = nu2;
            }
            red.sum3max(nu2, nw2, cr, mxu);
            s2 = s2 + 2.0 * cr + nu2 * nw2;
            ++q;
            if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max)
                break;
            // next row: tie-argmax of |u_q| over the unused rows
            const double thu = tie2 * mxu;
            int c = red.imin(tid < m && !used_row[tid] && cabs2(u) >= thu ? tid : m);
            if (c >= m) c = first_unused<NT>(used_row, m, red);
            i = min(c, m - 1);
        }
    } else if constexpr (PATH == 2) {
        // Several row and column entries per thread (j = tid + NT e, r = tid + NT e), kept in
        // registers.  The corrections read the history q' by q' for all of a thread's entries
        // at once (QB steps per batch, addresses clamped into the face, surplus terms masked
        // by a zero coefficient); b_q' = <w_q, w_q'> is formed by all threads from w_q in
        // registers, QB steps at a time, each wave's sums written to LDS and added up in a
        // fixed order; v is summed in the column pass as on the one-entry path.  After kBV
        // steps the face continues on the general path.
        constexpr int EM = kMultiE;
        constexpr int QB = MIXED ? 8 : 3;
        double2 *wpart = xbuf;   // [NW][64] per-wave partial sums of b
        FT *pivbuf = part;
        auto cmask = [](bool ok, FT a) {
            FT r;
            r.x = ok ? a.x : 0;
            r.y = ok ? a.y : 0;
            return r;
        };
        while (q < kBV) {
            FT *Wq = Wb + (int64_t)q * n;
            FT *Uq = Ub + (int64_t)q * m;
            FT v[EM];
#pragma unroll
            for (int e = 0; e < EM; ++e) v[e] = R[(int64_t)i * n + min(tid + NT * e, n - 1)];
            if (q > qL) stage_coef(Ub, m, i, q);
            {
                // row i of R - sum_{q'<q} u_q'[i] w_q'
                FT acc[EM];
#pragma unroll
                for (int e = 0; e < EM; ++e) acc[e] = czero<FT>();
                const int qm = min(q, qL);
                for (int qq = 0; qq < qm; ++qq) {
                    const FT c = Uh[qq * m + i];
#pragma unroll
                    for (int e = 0; e < EM; ++e) acc[e] = cfma(c, Wh[qq * n + min(tid + NT * e, n - 1)], acc[e]);
                }
                const int qc = min(q, qL + CL);
                for (int qq = qL; qq < qc; qq += QB) {
                    FT x[QB][EM];
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) {
                        const FT *wp = Wb + (int64_t)min(qq + qb, qc - 1) * n;
#pragma unroll
                        for (int e = 0; e < EM; ++e) x[qb][e] = wp[min(tid + NT * e, n - 1)];
                    }
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) {
                        const FT c = cmask(qq + qb < qc, cbuf[min(qq + qb, qc - 1) - qL]);
#pragma unroll
                        for (int e = 0; e < EM; ++e) acc[e] = cfma(c, x[qb][e], acc[e]);
                    }
                }
                for (int qq = qL + CL; qq < q; ++qq) {
                    const FT c = Ub[(int64_t)qq * m + i];
#pragma unroll
                    for (int e = 0; e < EM; ++e)
                        acc[e] = cfma(c, Wb[(int64_t)qq * n + min(tid + NT * e, n - 1)], acc[e]);
                }
#pragma unroll
                for (int e = 0; e < EM; ++e) v[e] = csub(v[e], acc[e]);
            }
            double mx = 0.0;
#pragma unroll
            for (int e = 0; e < EM; ++e)
                if (tid + NT * e < n) mx = fmax(mx, cabs2(v[e]));
            mx = red.max(mx);
            if (tid == 0) used_row[i] = 1;
            ++nused;
            if (sqrt(mx) <= zero_tol) {
                __syncthreads();
                int cand;
                if (q == 0) {
                    cand = first_nonzero_row<NT>(R, m, n, i + 1, zero_tol, red);
                    for (int r = i + 1 + tid; r < cand; r += NT) used_row[r] = 1;
                    nused += cand - (i + 1);
                } else {
                    cand = P.zero_batch ? zero_run() : first_unused<NT>(used_row, m, red);
                }
                if (cand >= m) {
                    fin = true;
                    break;
                }
                i = cand;
                continue;
            }
            const double thr = tie2 * mx;
            int jc = n;
#pragma unroll
            for (int e = EM - 1; e >= 0; --e)   // lowest own column at the threshold
                if (tid + NT * e < n && cabs2(v[e]) >= thr) jc = tid + NT * e;
            const int jp = min(red.imin(jc), n - 1);   // in range even for NaN rows
#pragma unroll
            for (int e = 0; e < EM; ++e)
                if (tid + NT * e == jp) pivbuf[0] = v[e];
            __syncthreads();
            const FT piv = pivbuf[0];
            FT cv[EM];
#pragma unroll
            for (int e = 0; e < EM; ++e) cv[e] = R[(int64_t)min(tid + NT * e, m - 1) * n + jp];
            double nw2 = 0.0;
#pragma unroll
            for (int e = 0; e < EM; ++e) {   // v <- w_q (zero beyond the face)
                const int j = tid + NT * e;
                if (j < n) {
                    const FT w = cdiv(v[e], piv);
                    v[e] = w;
                    Wq[j] = w;
                    if (q < qL) Wh[q * n + j] = w;
                    nw2 += cabs2(w);
                } else {
                    v[e] = czero<FT>();
                }
            }
            if (q > 0) {
                // b_q' = <w_q, w_q'>, 64 steps q' per round
                for (int qc0 = 0; qc0 < q; qc0 += 64) {
                    const int qn = min(64, q - qc0);
                    for (int qq = qc0; qq < qc0 + qn; qq += QB) {
                        FT x[QB][EM];
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb) {
                            const int qe = min(qq + qb, q - 1);
                            const FT *wp = qe < qL ? Wh + qe * n : Wb + (int64_t)qe * n;
#pragma unroll
                            for (int e = 0; e < EM; ++e) x[qb][e] = wp[min(tid + NT * e, n - 1)];
                        }
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb) {
                            double2 pb = make_double2(0.0, 0.0);
#pragma unroll
                            for (int e = 0; e < EM; ++e) pb = cfma(to_d2(v[e]), conj_d2(to_d2(x[qb][e])), pb);
                            pb.x = wave_sum(pb.x);
                            pb.y = wave_sum(pb.y);
                            if (lane == 0 && qq + qb < qc0 + qn) wpart[wave * 64 + qq + qb - qc0] = pb;
                        }
                    }
                    __syncthreads();
                    for (int t = tid; t < qn; t += NT) {
                        double2 sb = make_double2(0.0, 0.0);
                        for (int w = 0; w < NW; ++w) sb = cadd(sb, wpart[w * 64 + t]);
                        bvec[qc0 + t] = conj_d2(sb);
                    }
                    __syncthreads();
                }
            }
            if (q > qL) stage_coef(Wb, n, jp, q);
            // column jp of R - sum_{q'<q} w_q'[jp] u_q', and v = sum_{q'<q} conj(b_q') u_q'
            FT u[EM];
            double2 vv[EM];
            {
                FT acc[EM];
#pragma unroll
                for (int e = 0; e < EM; ++e) {
                    acc[e] = czero<FT>();
                    vv[e] = make_double2(0.0, 0.0);
                }
                const int qm = min(q, qL);
                for (int qq = 0; qq < qm; ++qq) {
                    const FT c = Wh[qq * n + jp];
                    const double2 bq = bvec[qq];
#pragma unroll
                    for (int e = 0; e < EM; ++e) {
                        const FT x = Uh[qq * m + min(tid + NT * e, m - 1)];
                        acc[e] = cfma(c, x, acc[e]);
                        vv[e] = cfma(bq, to_d2(x), vv[e]);
                    }
                }
                const int qc = min(q, qL + CL);
                for (int qq = qL; qq < qc; qq += QB) {
                    FT x[QB][EM];
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) {
                        const FT *up = Ub + (int64_t)min(qq + qb, qc - 1) * m;
#pragma unroll
                        for (int e = 0; e < EM; ++e) x[qb][e] = up[min(tid + NT * e, m - 1)];
                    }
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) {
                        const bool ok = qq + qb < qc;
                        const int qe = min(qq + qb, qc - 1);
                        const FT c = cmask(ok, cbuf[qe - qL]);
                        double2 bq = bvec[qe];
                        bq.x = ok ? bq.x : 0.0;
                        bq.y = ok ? bq.y : 0.0;
#pragma unroll
                        for (int e = 0; e < EM; ++e) {
                            acc[e] = cfma(c, x[qb][e], acc[e]);
                            vv[e] = cfma(bq, to_d2(x[qb][e]), vv[e]);
                        }
                    }
                }
                for (int qq = qL + CL; qq < q; ++qq) {
                    const FT c = Wb[(int64_t)qq * n + jp];
                    const double2 bq = bvec[qq];
#pragma unroll
                    for (int e = 0; e < EM; ++e) {
                        const FT x = Ub[(int64_t)qq * m + min(tid + NT * e, m - 1)];
                        acc[e] = cfma(c, x, acc[e]);
                        vv[e] = cfma(bq, to_d2(x), vv[e]);
                    }
                }
#pragma unroll
                for (int e = 0; e < EM; ++e) u[e] = csub(cv[e], acc[e]);
            }
            double nu2 = 0.0, cr = 0.0, mxu = -1.0;
#pragma unroll
            for (int e = 0; e < EM; ++e) {
                const int r = tid + NT * e;
                if (r < m) {
                    Uq[r] = u[e];
                    if (q < qL) Uh[q * m + r] = u[e];
                    const double a2 = cabs2(u[e]);
                    nu2 += a2;
                    const double2 ud = to_d2(u[e]);
                    cr += ud.x * vv[e].x + ud.y * vv[e].y;
                    if (!used_row[r]) mxu = fmax(mxu, a2);
                }
            }
            red.sum3max(nu2, nw2, cr, mxu);
            s2 = s2 + 2.0 * cr + nu2 * nw2;
            ++q;
            if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max) {
                fin = true;
                break;
            }
            // next row: tie-argmax of |u_q| over the unused rows
            const double thu = tie2 * mxu;
            int c = m;
#pragma unroll
            for (int e = EM - 1; e >= 0; --e) {
                const int r = tid + NT * e;
                if (r < m && !used_row[r] && cabs2(u[e]) >= thu) c = r;
            }
            c = red.imin(c);
            if (c >= m) c = first_unused<NT>(used_row, m, red);
            i = min(c, m - 1);
        }
    }
    if constexpr (PATH != 1)
    if (!fin)
    while (true) {
        FT *Wq = Wb + (int64_t)q * n;
        FT *Uq = Ub + (int64_t)q * m;
        // row i of R - sum_{q'<q} u_q'[i] w_q'
        double mx = 0.0;
        if (q > qL) stage_coef(Ub, m, i, q);
        if (splitw > 1) {
            const int s = tid / n, j = tid - s * n;
            if (s < splitw) {
                const int q0 = (int)((int64_t)q * s / splitw), q1 = (int)((int64_t)q * (s + 1) / splitw);
                part[tid] = hdot(Uh, Ub, m, i, Wh, Wb, n, j, q0, q1);
            }
            __syncthreads();
            if (tid < n) {
                FT v = R[(int64_t)i * n + tid];
                for (int t = 0; t < splitw; ++t) v = csub(v, part[t * n + tid]);
                Wq[tid] = v;
                mx = cabs2(v);
            }
        } else {
            for (int j = tid; j < n; j += NT) {
                FT v = csub(R[(int64_t)i * n + j], hdot(Uh, Ub, m, i, Wh, Wb, n, j, 0, q));
                Wq[j] = v;
                mx = fmax(mx, cabs2(v));
            }
        }
        mx = red.max(mx);
        if (tid == 0) used_row[i] = 1;
        ++nused;
        if (sqrt(mx) <= zero_tol) {
            __syncthreads();
            int cand;
            if (q == 0) {
                cand = first_nonzero_row<NT>(R, m, n, i + 1, zero_tol, red);
                for (int r = i + 1 + tid; r < cand; r += NT) used_row[r] = 1;
                nused += cand - (i + 1);
            } else {
                cand = first_unused<NT>(used_row, m, red);
            }
            if (cand >= m) break;
            i = cand;
            continue;
        }
        const double thr = tie2 * mx;
        int jc = n;
        for (int j = tid; j < n; j += NT)
            if (cabs2(Wq[j]) >= thr) {
                jc = j;
                break;
            }
        const int jp = min(red.imin(jc), n - 1);   // in range even for NaN rows
        const FT piv = Wq[jp];
        __syncthreads();
        double nw2 = 0.0, nu2 = 0.0;
        for (int j = tid; j < n; j += NT) {
            const FT w = cdiv(Wq[j], piv);
            Wq[j] = w;
            if (q < qL) Wh[q * n + j] = w;
            nw2 += cabs2(w);
        }
        __syncthreads();
        // column jp of R - sum_{q'<q} w_q'[jp] u_q'
        if (q > qL) stage_coef(Wb, n, jp, q);
        if (splitu > 1) {
            const int s = tid / m, r = tid - s * m;
            if (s < splitu) {
                const int q0 = (int)((int64_t)q * s / splitu), q1 = (int)((int64_t)q * (s + 1) / splitu);
                part[tid] = hdot(Wh, Wb, n, jp, Uh, Ub, m, r, q0, q1);
            }
            __syncthreads();
            if (tid < m) {
                FT u = R[(int64_t)tid * n + jp];
                for (int t = 0; t < splitu; ++t) u = csub(u, part[t * m + tid]);
                Uq[tid] = u;
                if (q < qL) Uh[q * m + tid] = u;
                nu2 += cabs2(u);
            }
        } else {
            for (int r = tid; r < m; r += NT) {
                const FT u = csub(R[(int64_t)r * n + jp], hdot(Wh, Wb, n, jp, Uh, Ub, m, r, 0, q));
                Uq[r] = u;
                if (q < qL) Uh[q * m + r] = u;
                nu2 += cabs2(u);
            }
        }
        __syncthreads();
        // sum_{q'<q} Re(<u_q, u_q'> <w_q, w_q'>) in FP64
        const FT *uc = q < qL ? Uh + (int64_t)q * m : Uq;
        const FT *wc = q < qL ? Wh + (int64_t)q * n : Wq;
        double cr = 0.0;
        constexpr int CR = NT >= 1024 ? 3 : kCurRegs;
        if (m <= 64 * CR && n <= 64 * CR) {
            // u_q, w_q held in registers; QPI q' per wave iteration, all loads issued first
            double2 ucr[CR], wcr[CR];
#pragma unroll
            for (int t = 0; t < CR; ++t) {
                const int r = lane + 64 * t;
                ucr[t] = r < m ? to_d2(uc[r]) : make_double2(0.0, 0.0);
                wcr[t] = r < n ? to_d2(wc[r]) : make_double2(0.0, 0.0);
            }
            constexpr int QPI = NT >= 1024 ? 1 : 2;   // q' per wave iteration (registers)
            for (int q0 = wave; q0 < q; q0 += QPI * NW) {
                FT uu[QPI][CR], ww[QPI][CR];
#pragma unroll
                for (int g = 0; g < QPI; ++g) {
                    const int qg = q0 + g * NW;
                    const bool ok = qg < q;
                    const FT *up = qg < qL ? Uh + (int64_t)qg * m : Ub + (int64_t)qg * m;
                    const FT *wp = qg < qL ? Wh + (int64_t)qg * n : Wb + (int64_t)qg * n;
#pragma unroll
                    for (int t = 0; t < CR; ++t) {
                        const int r = lane + 64 * t;
                        uu[g][t] = (ok && r < m) ? up[r] : czero<FT>();
                        ww[g][t] = (ok && r < n) ? wp[r] : czero<FT>();
                    }
                }
#pragma unroll
                for (int g = 0; g < QPI; ++g) {
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                    for (int t = 0; t < CR; ++t) {
                        double2 v = cmulc(ucr[t], to_d2(uu[g][t]));
                        a0 += v.x;
                        a1 += v.y;
                        v = cmulc(wcr[t], to_d2(ww[g][t]));
                        a2 += v.x;
                        a3 += v.y;
                    }
                    a0 = wave_sum(a0);
                    a1 = wave_sum(a1);
                    a2 = wave_sum(a2);
                    a3 = wave_sum(a3);
                    if (q0 + g * NW < q) cr += a0 * a2 - a1 * a3;
                }
            }
        } else
        for (int qq = wave; qq < q; qq += NW) {
            const FT *up = qq < qL ? Uh + (int64_t)qq * m : Ub + (int64_t)qq * m;
            const FT *wp = qq < qL ? Wh + (int64_t)qq * n : Wb + (int64_t)qq * n;
            double ur = 0.0, ui = 0.0, wr = 0.0, wi = 0.0;
            for (int r = lane; r < m; r += 64) {
                const double2 v = cmulc(to_d2(uc[r]), to_d2(up[r]));
                ur += v.x;
                ui += v.y;
            }
            for (int j = lane; j < n; j += 64) {
                const double2 v = cmulc(to_d2(wc[j]), to_d2(wp[j]));
                wr += v.x;
                wi += v.y;
            }
            ur = wave_sum(ur);
            ui = wave_sum(ui);
            wr = wave_sum(wr);
            wi = wave_sum(wi);
            cr += ur * wr - ui * wi;
        }
        if (lane != 0) cr = 0.0;
        red.sum3(nu2, nw2, cr);
        s2 = s2 + 2.0 * cr + nu2 * nw2;
        ++q;
        if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max)
            break;
        i = pick_unused<NT>(Uq, used_row, m, tie2, red);
    }
    if (tid == 0) {
        bd.st[b].rho = q;
        bd.st[b].aca_ticks += wall_clock64() - t_start;
    }
}

// ---------------------------------------------------------------------------------------
// Expand phase (kind 2): one 32 x 32 tile of H_l = U W^T per wave, written over R, with the
// tile's max |H|^2, sum |H|^2 and Gram partials <H_l, H_p>.  Lane (rg, cg) = (lane / 8,
// lane % 8) owns the sixteen entries (rg + 8 a, cg + 8 e), a, e < 4: each factor step
// reads four U and four W values from LDS for sixteen complex products, and for each (a, e)
// the wave touches eight rows of eight consecutive elements, so every load and store of the
// face pool covers whole row segments.  The Gram row streams the previous faces with sixteen
// loads in flight per lane and one wave reduction per face, with no barrier.
template <bool MIXED>
__global__ void __launch_bounds__(64) far_expand_kernel(FarBatchDev bd, const FarActive *act) {
    using FT = face_t<MIXED>;
    constexpr int T = kFarTile;
    constexpr int QC = 8;   // factor steps staged in LDS per pass
    static_assert(T == 32, "the lane layout covers 32 x 32 tiles");
    const int64_t c = blockIdx.x;
    const int a = bd.map_tile[c];
    const FarActive A = act[a];
    const int b = A.b;
    const int rho = bd.st[b].rho, ell = bd.st[b].ell;
    if (rho == 0) return;
    const FarBlockDev B = bd.blk[b];
    const int m = B.m, n = B.n;
    const int t = (int)(c - A.tile0), ntj = (n + T - 1) / T;
    const int i0 = (t / ntj) * T, j0 = (t % ntj) * T;
    const int lane = threadIdx.x, rg = lane >> 3, cg = lane & 7;
    const FT *Ub = reinterpret_cast<const FT *>(bd.uw) + B.uw_off;
    const FT *Wb = Ub + (int64_t)B.rho_max * m;
    // tile origin in the face (row-major m x n)
    const int64_t org = (int64_t)i0 * n + j0;
    FT *H = reinterpret_cast<FT *>(bd.hpool) + A.hslot + org;
    const FT *hp = reinterpret_cast<const FT *>(bd.hpool) + org;

    __shared__ FT Us[QC][T];
    __shared__ FT Ws[QC][T];
    FT acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[x][e] = czero<FT>();
    for (int q0 = 0; q0 < rho; q0 += QC) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < QC * T / 64; ++e) {
            const int id = lane + 64 * e, qq = id >> 5, ii = id & 31;
            const bool qv = q0 + qq < rho;
            Us[qq][ii] = (qv && i0 + ii < m) ? Ub[(int64_t)(q0 + qq) * m + i0 + ii] : czero<FT>();
            Ws[qq][ii] = (qv && j0 + ii < n) ? Wb[(int64_t)(q0 + qq) * n + j0 + ii] : czero<FT>();
        }
        __syncthreads();
        const int nq = min(QC, rho - q0);
        for (int qq = 0; qq < nq; ++qq) {
            FT u[4], w[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) u[x] = Us[qq][rg + 8 * x];
#pragma unroll
            for (int e = 0; e < 4; ++e) w[e] = Ws[qq][cg + 8 * e];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[x][e] = cfma(u[x], w[e], acc[x][e]);
        }
    }
    // entry offsets from the tile origin; entries outside the face are masked
    bool ok[4][4];
    int off[4][4];
    double mx = 0.0, s = 0.0;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = rg + 8 * x, cc = cg + 8 * e;
            ok[x][e] = i0 + r < m && j0 + cc < n;
            off[x][e] = r * n + cc;
            if (ok[x][e]) {
                H[off[x][e]] = acc[x][e];
                const double a2 = cabs2(acc[x][e]);
                mx = fmax(mx, a2);
                s += a2;
            }
        }
    double *out = bd.part + (A.tile0 + t) * (int64_t)far_part_stride(bd.rcap);
    mx = wave_max(mx);
    s = wave_sum(s);
    if (lane == 0) {
        out[0] = mx;
        out[1] = s;
    }
    const int64_t *hs = bd.hs + (int64_t)b * bd.rcap;
    for (int p = 0; p < ell; ++p) {
        const FT *hq = hp + hs[p];
        FT v[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int e = 0; e < 4; ++e) v[x][e] = ok[x][e] ? hq[off[x][e]] : czero<FT>();
        double gr = 0.0, gi = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double2 g = cmulc(to_d2(acc[x][e]), to_d2(v[x][e]));
                gr += g.x;
                gi += g.y;
            }
        gr = wave_sum(gr);
        gi = wave_sum(gi);
        if (lane == 0) {
            out[2 + 2 * p] = gr;
            out[3 + 2 * p] = gi;
        }
    }
}

// Gram row <H_l, H_p> (p < l) of a small face (kinds 0/1, H_l already stored by the ACA
// phase), one workgroup per face, written as the face's single partial row.
__global__ void __launch_bounds__(256) far_gram_small_kernel(FarBatchDev bd, const FarActive *act) {
    const FarActive A = act[blockIdx.x];
    const int b = A.b;
    const int rho = bd.st[b].rho, ell = bd.st[b].ell;
    if (rho == 0) return;
    const FarBlockDev B = bd.blk[b];
    const int mn = B.m * B.n, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    __shared__ int64_t hsl[kMaxRcap];
    __shared__ double red8[8][4];
    for (int p = tid; p < ell; p += 256) hsl[p] = bd.hs[(int64_t)b * bd.rcap + p];
    __syncthreads();
    double *out = bd.part + A.tile0 * (int64_t)far_part_stride(bd.rcap);
    auto run = [&](auto tag) {
        using FT = decltype(tag);
        const FT *hp = reinterpret_cast<const FT *>(bd.hpool);
        const FT *H = hp + A.hslot;
        for (int p0 = 0; p0 < ell; p0 += 4) {
            const int np = min(4, ell - p0);
            double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int idx = tid; idx < mn; idx += 256) {
                const double2 h = to_d2(H[idx]);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
                    if (tt < np) {
                        const double2 v = cmulc(h, to_d2(hp[hsl[p0 + tt] + idx]));
                        g[2 * tt] += v.x;
                        g[2 * tt + 1] += v.y;
                    }
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) g[v] = wave_sum(g[v]);
            __syncthreads();
            if (lane == 0)
#pragma unroll
                for (int v = 0; v < 8; ++v) red8[v][wave] = g[v];
            __syncthreads();
            if (tid < 2 * np)
                out[2 + 2 * p0 + tid] = (red8[tid][0] + red8[tid][1]) + (red8[tid][2] + red8[tid][3]);
        }
    };
    if (bd.mixed) run(float2{});
    else run(double2{});
}

// ---------------------------------------------------------------------------------------
// Tail phase: one workgroup of NT threads per active block.
template <int KERNEL, bool DENSE, bool MIXED, int NT>
__global__ void __launch_bounds__(NT)
    far_tail_kernel(GeoDev g, FreqDev f, AcaParams P, FarBatchDev bd, const FarActive *act,
                    int nlarge) {
    using FT = face_t<MIXED>;
    constexpr int NW = NT / 64;
    const int a = blockIdx.x;
    const FarActive A = act[a];
    const int b = A.b;
    const FarBlockDev B = bd.blk[b];
    FarStateDev S = bd.st[b];
    const int L = f.L, rcap = bd.rcap, m = B.m, n = B.n;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);
    const FT *hp = reinterpret_cast<const FT *>(bd.hpool);
    const FT *H = hp + A.hslot;
    double2 *fg = bd.fgpool;

    __shared__ unsigned char used_k[kMaxLds];
    __shared__ int64_t fsl[kMaxRcap], hsl[kMaxRcap];
    __shared__ double2 gsh[kMaxRcap], hpiv_p[kMaxRcap], coefs[kMaxRcap];
    __shared__ double redbuf[8 * NW + 4];
    Red<NT> red{redbuf};

    for (int kk = tid; kk < L; kk += NT) used_k[kk] = bd.usedk[(int64_t)b * L + kk];
    for (int p = tid; p < S.ell; p += NT) {
        fsl[p] = bd.fs[(int64_t)b * rcap + p];
        hsl[p] = bd.hs[(int64_t)b * rcap + p];
    }
    __syncthreads();
    if (tid == 0) used_k[S.k] = 1;
    S.nused_k += 1;
    const int rho = S.rho;
    bool done = false;
    if (rho == 0) {
        S.zero_faces += 1;
        S.zero_run += 1;
        __syncthreads();
        if (S.zero_run >= 3 || S.nused_k >= L) done = true;
        else S.k = first_unused<NT>(used_k, L, red);
    } else {
        S.zero_run = 0;
        const int ell = S.ell;
        double mxh, h2;
        int pidx;
        if (a < nlarge) {
            // reduce the expand partials (fixed order) and locate the pivot
            const int PS = far_part_stride(rcap);
            const double *pt = bd.part + A.tile0 * (int64_t)PS;
            double mx = 0.0, s = 0.0;
            for (int t = tid; t < A.ntile; t += NT) {
                mx = fmax(mx, pt[(int64_t)t * PS]);
                s += pt[(int64_t)t * PS + 1];
            }
            red.maxsum(mx, s);
            mxh = mx;
            h2 = s;
            for (int p = tid; p < ell; p += NT) {
                double gr = 0.0, gi = 0.0;
                for (int t = 0; t < A.ntile; ++t) {
                    gr += pt[(int64_t)t * PS + 2 + 2 * p];
                    gi += pt[(int64_t)t * PS + 3 + 2 * p];
                }
                gsh[p] = make_double2(gr, gi);
                fg[A.fgslot + L + p] = gsh[p];
            }
            if (tid == 0) fg[A.fgslot + L + ell] = make_double2(h2, 0.0);
            const double thh = tie2 * mxh;
            int tc = 0x7fffffff;
            for (int t = tid; t < A.ntile; t += NT)
                if (pt[(int64_t)t * PS] >= thh) {
                    tc = t;
                    break;
                }
            tc = red.imin(tc);
            if (tc >= A.ntile) tc = 0;   // no tile compares (NaN)
            const int ntj = (n + kFarTile - 1) / kFarTile;
            const int64_t lo = (int64_t)(tc / ntj) * kFarTile * n;
            const int64_t hi = min((int64_t)m, (int64_t)(tc / ntj + 1) * kFarTile) * n;
            int pc = 0x7fffffff;
            for (int64_t idx = lo + tid; idx < hi; idx += NT)
                if (cabs2(H[idx]) >= thh) {
                    pc = (int)idx;
                    break;
                }
            pidx = (int)min((int64_t)red.imin(pc), hi - 1);
            if (P.pivot_index) {
                // eq. (index): row i of the largest sum_q |U'(q, i)| (U' = U_bar Sigma after the
                // recompression), then the largest entry of row i of H_l (same tie rule)
                const FT *Uf = reinterpret_cast<const FT *>(bd.uw) + B.uw_off;
                double best = 0.0;
                for (int i = tid; i < m; i += NT) {
                    double sa = 0.0;
                    for (int q = 0; q < rho; ++q) sa += sqrt(cabs2(Uf[(int64_t)q * m + i]));
                    best = fmax(best, sa * sa);
                }
                best = red.max(best);
                int ic = 0x7fffffff;
                for (int i = tid; i < m; i += NT) {
                    double sa = 0.0;
                    for (int q = 0; q < rho; ++q) sa += sqrt(cabs2(Uf[(int64_t)q * m + i]));
                    if (sa * sa >= tie2 * best) {
                        ic = i;
                        break;
                    }
                }
                ic = min(red.imin(ic), m - 1);
                double rb = 0.0;
                for (int j = tid; j < n; j += NT) rb = fmax(rb, cabs2(H[(int64_t)ic * n + j]));
                rb = red.max(rb);
                int jc = 0x7fffffff;
                for (int j = tid; j < n; j += NT)
                    if (cabs2(H[(int64_t)ic * n + j]) >= tie2 * rb) {
                        jc = j;
                        break;
                    }
                jc = min(red.imin(jc), n - 1);
                pidx = ic * n + jc;
            }
        } else {
            mxh = S.mxh;
            h2 = S.h2;
            pidx = S.pidx;
            const double *pt = bd.part + A.tile0 * (int64_t)far_part_stride(rcap);
            for (int p = tid; p < ell; p += NT) {
                gsh[p] = make_double2(pt[2 + 2 * p], pt[3 + 2 * p]);
                fg[A.fgslot + L + p] = gsh[p];
            }
            if (tid == 0) fg[A.fgslot + L + ell] = make_double2(h2, 0.0);
        }
        (void)mxh;
        const double2 hpiv = to_d2(H[pidx]);
        const int ip = pidx / n, jpv = pidx - ip * n;
        for (int p = tid; p < ell; p += NT) hpiv_p[p] = to_d2(hp[hsl[p] + pidx]);
        __syncthreads();
        // frequency fibre through the pivot (FP64)
        double2 *fl_ = fg + A.fgslot;
        for (int kk = tid; kk < L; kk += NT) {
            double2 e = fibre_entry<KERNEL, DENSE>(g, f, bd.dense, B, ip, jpv, kk);
#pragma unroll 4
            for (int p = 0; p < ell; ++p) e = csub(e, cmul(hpiv_p[p], fg[fsl[p] + kk]));
            fl_[kk] = cdiv(e, hpiv);
        }
        __syncthreads();
        // eq. (norm) update
        double c3 = 0.0, f2 = 0.0, fmx = 0.0;
        for (int p = wave; p < ell; p += NW) {
            double dr = 0.0, di = 0.0;
            for (int kk = lane; kk < L; kk += 64) {
                const double2 t = cmulc(fl_[kk], fg[fsl[p] + kk]);
                dr += t.x;
                di += t.y;
            }
            dr = wave_sum(dr);
            di = wave_sum(di);
            c3 += gsh[p].x * dr - gsh[p].y * di;
        }
        if (lane != 0) c3 = 0.0;
        for (int kk = tid; kk < L; kk += NT) {
            const double a2 = cabs2(fl_[kk]);
            f2 += a2;
            fmx = fmax(fmx, a2);
        }
        fmx = red.max(fmx);
        double unused0 = 0.0;
        red.sum3(c3, f2, unused0);
        S.norm2 = S.norm2 + 2.0 * c3 + h2 * f2;
        S.scale = fmax(S.scale, sqrt(cabs2(hpiv)) * sqrt(fmx));
        if (tid == 0) {
            bd.cmeta[(int64_t)B.out_idx * rcap + ell] = CrossMeta{S.k, ip, jpv, rho};
            bd.hs[(int64_t)b * rcap + ell] = A.hslot;
            bd.fs[(int64_t)b * rcap + ell] = A.fgslot;
            fsl[ell] = A.fgslot;
        }
        S.sum_rho += rho;
        S.ell = ell + 1;
        if (sqrt(h2 * f2) <= P.eps * sqrt(fmax(S.norm2, 0.0))) done = true;
        else if (S.nused_k >= L) done = true;
        else if (S.ell >= rcap) {
            S.capped = 1;
            done = true;
        } else {
            S.k = pick_unused<NT>(fl_, used_k, L, tie2, red);
        }
    }
    if (!done) {
        // residual coefficients and |C^(l)(:,:,k)|_F^2 of the next face
        __syncthreads();
        const int ell = S.ell;
        double2 isc = make_double2(1.0, 0.0);
        if (MIXED) isc = inv_scale(f, B, S.k);
        for (int p = tid; p < ell; p += NT) {
            coefs[p] = cmul(fg[fsl[p] + S.k], isc);
            bd.coef[(int64_t)b * rcap + p] = coefs[p];
        }
        __syncthreads();
        double part = 0.0;
        for (int x = tid; x < ell; x += NT)
            for (int y = 0; y < ell; ++y) {
                const double2 gxy = x >= y ? fg[fsl[x] + L + y] : conj_d2(fg[fsl[y] + L + x]);
                part += cmul(cmulc(coefs[x], coefs[y]), gxy).x;
            }
        S.ref2 = fmax(red.sum(part), 0.0);
        S.zero_tol = P.delta * S.scale * (MIXED ? sqrt(cabs2(isc)) : 1.0);
    }
    S.done = done ? 1 : 0;
    if (tid == 0) {
        bd.st[b] = S;
        bd.status[2 * a] = (rho > 0 ? 1 : 0) | (done ? 2 : 0);
        bd.status[2 * a + 1] = rho;
        if (done) {
            FarMeta mt;
            mt.rank = S.ell;
            mt.sum_rho = S.sum_rho;
            mt.capped = S.capped;
            mt.zero_faces = S.zero_faces;
            mt.aca_ticks = S.aca_ticks;
            mt.norm2 = S.norm2;
            bd.meta[B.out_idx] = mt;
        }
    }
    __syncthreads();
    for (int kk = tid; kk < L; kk += NT) bd.usedk[(int64_t)b * L + kk] = used_k[kk];
}

// ---------------------------------------------------------------------------------------
// Factors of accepted crosses -> arena (U: rho x m, then W: rho x n), kFarCopyChunk elements
// per workgroup with all loads of a thread issued before its stores.
template <class FT>
__global__ void __launch_bounds__(256) far_copy_kernel(FarBatchDev bd, const FarCopy *cp,
                                                       FT *arena0, FT *arena1, int64_t *cross_off) {
    constexpr int PER = kFarCopyChunk / 256;
    const FarCopy C = cp[blockIdx.x];
    FT *arena = C.which ? arena1 : arena0;
    const FarBlockDev B = bd.blk[C.b];
    const FT *Ub = reinterpret_cast<const FT *>(bd.uw) + B.uw_off;
    const FT *Wb = Ub + (int64_t)B.rho_max * B.m;
    const int64_t nu = (int64_t)C.rho * B.m, tot = nu + (int64_t)C.rho * B.n;
    const int64_t e0 = (int64_t)C.chunk * kFarCopyChunk + threadIdx.x;
    FT v[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int64_t e = e0 + 256 * t;
        FT x = czero<FT>();
        if (e < nu) x = Ub[e];
        else if (e < tot) x = Wb[e - nu];
        v[t] = x;
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int64_t e = e0 + 256 * t;
        if (e < tot) arena[C.off + e] = v[t];
    }
    if (C.chunk == 0 && threadIdx.x == 0) cross_off[(int64_t)B.out_idx * bd.rcap + C.p] = C.off;
}

// Fibres of finished blocks -> fibre arena (rank x L, contiguous per block).
__global__ void __launch_bounds__(256) far_gather_kernel(FarBatchDev bd, const FarGather *gt,
                                                         double2 *fib0, double2 *fib1, int64_t *fib_off) {
    const FarGather G = gt[blockIdx.x];
    double2 *fib_arena = G.which ? fib1 : fib0;
    const FarBlockDev B = bd.blk[G.b];
    const int L = bd.L;
    for (int p = 0; p < G.rank; ++p) {
        const int64_t src = bd.fs[(int64_t)G.b * bd.rcap + p];
        for (int kk = threadIdx.x; kk < L; kk += 256)
            fib_arena[G.off + (int64_t)p * L + kk] = bd.fgpool[src + kk];
    }
    if (threadIdx.x == 0) fib_off[B.out_idx] = G.off;
}

// ---------------------------------------------------------------------------------------
void launch_far_map(const FarBatchDev &bd, const FarActive *act, int nact, int nlarge,
                    hipStream_t st) {
    if (nact <= 0) return;
    far_map_kernel<<<nact, 256, 0, st>>>(bd, act, nact, nlarge);
}

template <int K, bool D, bool MX>
static void face_dispatch(const GeoDev &g, const FreqDev &f, const FarBatchDev &bd,
                          const FarActive *act, int64_t nchunk, hipStream_t st) {
    far_face_kernel<K, D, MX><<<(unsigned)nchunk, kFarChunk, 0, st>>>(g, f, bd, act);
}

void launch_far_face(int kernel, const GeoDev &g, const FreqDev &f, const FarBatchDev &bd,
                     const FarActive *act, int64_t nchunk, hipStream_t st) {
    if (nchunk <= 0) return;
    if (bd.dense) face_dispatch<0, true, false>(g, f, bd, act, nchunk, st);
    else if (kernel < 0) {
        if (bd.mixed) face_dispatch<-1, false, true>(g, f, bd, act, nchunk, st);
        else face_dispatch<-1, false, false>(g, f, bd, act, nchunk, st);
    } else if (!bd.mixed) {
        if (kernel == 0) face_dispatch<0, false, false>(g, f, bd, act, nchunk, st);
        else if (kernel == 1) face_dispatch<1, false, false>(g, f, bd, act, nchunk, st);
        else if (kernel == 3) face_dispatch<3, false, false>(g, f, bd, act, nchunk, st);
        else if (kernel == 4) face_dispatch<4, false, false>(g, f, bd, act, nchunk, st);
        else if (kernel == 5) face_dispatch<5, false, false>(g, f, bd, act, nchunk, st);
        else face_dispatch<2, false, false>(g, f, bd, act, nchunk, st);
    } else {
        if (kernel == 0) face_dispatch<0, false, true>(g, f, bd, act, nchunk, st);
        else if (kernel == 1) face_dispatch<1, false, true>(g, f, bd, act, nchunk, st);
        else face_dispatch<2, false, true>(g, f, bd, act, nchunk, st);
    }
}

template <bool MX, int PATH>
static void large_dispatch(int threads, const AcaParams &P, const FarBatchDev &bd,
                           const FarActive *act, int nact, hipStream_t st) {
    // large faces: one face per CU with 1024 or 512 threads and ~100 KB of LDS history, or
    // 256 threads with 59 KB (one entry per thread) or 32 KB, two per CU
    if constexpr (PATH == 2) {
        far_aca_large_kernel<512, MX, 106496, 2><<<nact, 512, 0, st>>>(P, bd, act);
    } else {
        if (threads >= 1024)
            far_aca_large_kernel<1024, MX, 90112, PATH><<<nact, 1024, 0, st>>>(P, bd, act);
        else if (threads >= 512)
            far_aca_large_kernel<512, MX, 106496, PATH><<<nact, 512, 0, st>>>(P, bd, act);
        else   // one-entry path: smaller flag / coefficient / Gram arrays leave ~59 KB of history
            far_aca_large_kernel<256, MX, PATH == 1 ? 60800 : 32768, PATH><<<nact, 256, 0, st>>>(P, bd, act);
    }
}

template <bool MX>
static void aca_dispatch(int path, int threads, const AcaParams &P, const FarBatchDev &bd,
                         const FarActive *act, int nact, hipStream_t st) {
    if (path == 1) large_dispatch<MX, 1>(threads, P, bd, act, nact, st);
    else if (path == 2) large_dispatch<MX, 2>(threads, P, bd, act, nact, st);
    else large_dispatch<MX, 0>(threads, P, bd, act, nact, st);
}

template <bool MX>
static void aca_small_dispatch(int mnmax, int threads, const AcaParams &P, const FarBatchDev &bd,
                               const FarActive *act, int nact, hipStream_t st) {
    if (mnmax <= 576 && threads <= 64)
        far_aca_small_kernel<64, MX, 576, 64><<<nact, 64, 0, st>>>(P, bd, act);
    else if (mnmax <= 1024 && threads <= 64)
        far_aca_small_kernel<64, MX, 1024, 64><<<nact, 64, 0, st>>>(P, bd, act);
    else if (mnmax <= 1024)
        far_aca_small_kernel<128, MX, 1024, 64><<<nact, 128, 0, st>>>(P, bd, act);
    else if (mnmax <= 2304 && threads <= 64)
        far_aca_small_kernel<64, MX, 2304, 96><<<nact, 64, 0, st>>>(P, bd, act);
    else if (mnmax <= 2304 && threads <= 128)
        far_aca_small_kernel<128, MX, 2304, 96><<<nact, 128, 0, st>>>(P, bd, act);
    else if (mnmax <= 2304)
        far_aca_small_kernel<256, MX, 2304, 96><<<nact, 256, 0, st>>>(P, bd, act);
    else
        far_aca_small_kernel<512, MX, 4096, 128><<<nact, 512, 0, st>>>(P, bd, act);
}

void launch_far_aca(int path, int threads, const AcaParams &P, const FarBatchDev &bd,
                    const FarActive *act, int nact, hipStream_t st) {
    if (nact <= 0) return;
    if (bd.mixed) aca_dispatch<true>(path, threads, P, bd, act, nact, st);
    else aca_dispatch<false>(path, threads, P, bd, act, nact, st);
}

void launch_far_aca_small(int mnmax, int threads, const AcaParams &P, const FarBatchDev &bd,
                          const FarActive *act, int nact, hipStream_t st) {
    if (nact <= 0) return;
    if (bd.mixed) aca_small_dispatch<true>(mnmax, threads, P, bd, act, nact, st);
    else aca_small_dispatch<false>(mnmax, threads, P, bd, act, nact, st);
}

void launch_far_expand(const FarBatchDev &bd, const FarActive *act, int64_t ntile, hipStream_t st) {
    if (ntile <= 0) return;
    if (bd.mixed) far_expand_kernel<true><<<(unsigned)ntile, 64, 0, st>>>(bd, act);
    else far_expand_kernel<false><<<(unsigned)ntile, 64, 0, st>>>(bd, act);
}

void launch_far_gram_small(const FarBatchDev &bd, const FarActive *act, int nact, hipStream_t st) {
    if (nact <= 0) return;
    far_gram_small_kernel<<<nact, 256, 0, st>>>(bd, act);
}

template <int K, bool D, bool MX>
static void tail_dispatch(const GeoDev &g, const FreqDev &f, const AcaParams &P,
                          const FarBatchDev &bd, const FarActive *act, int nact, int nlarge,
                          hipStream_t st) {
    // two waves per block: the fibre of L <= 128 frequencies is one entry per thread, and twice
    // as many blocks share a CU as with four waves
    constexpr int kTailThreads = 128;
    far_tail_kernel<K, D, MX, kTailThreads><<<nact, kTailThreads, 0, st>>>(g, f, P, bd, act, nlarge);
}

void launch_far_tail(int kernel, const GeoDev &g, const FreqDev &f, const AcaParams &P,
                     const FarBatchDev &bd, const FarActive *act, int nact, int nlarge,
                     hipStream_t st) {
    if (nact <= 0) return;
    if (bd.dense) tail_dispatch<0, true, false>(g, f, P, bd, act, nact, nlarge, st);
    else if (kernel < 0) {
        if (bd.mixed) tail_dispatch<-1, false, true>(g, f, P, bd, act, nact, nlarge, st);
        else tail_dispatch<-1, false, false>(g, f, P, bd, act, nact, nlarge, st);
    } else if (!bd.mixed) {
        if (kernel == 0) tail_dispatch<0, false, false>(g, f, P, bd, act, nact, nlarge, st);
        else if (kernel == 1) tail_dispatch<1, false, false>(g, f, P, bd, act, nact, nlarge, st);
        else if (kernel == 3) tail_dispatch<3, false, false>(g, f, P, bd, act, nact, nlarge, st);
        else if (kernel == 4) tail_dispatch<4, false, false>(g, f, P, bd, act, nact, nlarge, st);
        else if (kernel == 5) tail_dispatch<5, false, false>(g, f, P, bd, act, nact, nlarge, st);
        else tail_dispatch<2, false, false>(g, f, P, bd, act, nact, nlarge, st);
    } else {
        if (kernel == 0) tail_dispatch<0, false, true>(g, f, P, bd, act, nact, nlarge, st);
        else if (kernel == 1) tail_dispatch<1, false, true>(g, f, P, bd, act, nact, nlarge, st);
        else tail_dispatch<2, false, true>(g, f, P, bd, act, nact, nlarge, st);
    }
}

void launch_far_copy(const FarBatchDev &bd, const FarCopy *c, int n, void *const arena[2],
                     int64_t *cross_off, hipStream_t st) {
    if (n <= 0) return;
    if (bd.mixed)
        far_copy_kernel<float2><<<n, 256, 0, st>>>(bd, c, reinterpret_cast<float2 *>(arena[0]),
                                                  reinterpret_cast<float2 *>(arena[1]), cross_off);
    else
        far_copy_kernel<double2><<<n, 256, 0, st>>>(bd, c, reinterpret_cast<double2 *>(arena[0]),
                                                   reinterpret_cast<double2 *>(arena[1]), cross_off);
}

void launch_far_gather(const FarBatchDev &bd, const FarGather *gt, int n, double2 *const fib_arena[2],
                       int64_t *fib_off, hipStream_t st) {
    if (n <= 0) return;
    far_gather_kernel<<<n, 256, 0, st>>>(bd, gt, fib_arena[0], fib_arena[1], fib_off);
}


// ---------------------------------------------------------------------------------------
// Test hook: mixed-precision face entries of one block, multiplied back by c_k in FP64.
template <int KERNEL>
__global__ void eval_far_mixed_kernel(GeoDev g, FreqDev f, FarBlockDev B, int64_t n,
                                      const int32_t *il, const int32_t *jl, const int32_t *kk,
                                      double2 *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float2 e = face_entry<KERNEL, false, float2>(g, f, nullptr, B, il[t], jl[t], kk[t]);
    const double2 ic = inv_scale(f, B, kk[t]);   // 1 / c_k
    const double den = ic.x * ic.x + ic.y * ic.y;
    const double er = e.x, ei = e.y;
    out[t] = make_double2((er * ic.x + ei * ic.y) / den, (ei * ic.x - er * ic.y) / den);
}

void launch_eval_far_mixed(int kernel, const GeoDev &g, const FreqDev &f, const FarBlockDev &B,
                           int64_t n, const int32_t *il, const int32_t *jl, const int32_t *k,
                           double2 *out, hipStream_t st) {
    if (n <= 0) return;
    const unsigned nb = (unsigned)((n + 127) / 128);
    if (kernel == 0) eval_far_mixed_kernel<0><<<nb, 128, 0, st>>>(g, f, B, n, il, jl, k, out);
    else if (kernel == 1) eval_far_mixed_kernel<1><<<nb, 128, 0, st>>>(g, f, B, n, il, jl, k, out);
    else eval_far_mixed_kernel<2><<<nb, 128, 0, st>>>(g, f, B, n, il, jl, k, out);
}

}  // namespace gaca
