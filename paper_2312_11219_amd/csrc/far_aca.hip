// 3D-ACA of far (admissible) blocks: Algorithm 1 of the paper with ACA faces and the
// dense-expansion pivot, one workgroup per block, FP64 or mixed precision.
//
// Per face l (frequency k_l):
//   residual face R = ENTRY(:, :, k) - sum_{p < l} f_p[k] H_p   (previous dense faces H_p)
//   partial-pivot ACA of R  -> u_q, w_q, stop when |u||w| <= eps_aca sqrt(|C(:,:,k)|^2 + |S|^2)
//   H_l = sum_q u_q w_q^T, pivot (i_l, j_l) = tie-argmax |H_l|
//   fibre f_l[k'] = (ENTRY(i_l, j_l, k') - sum_p H_p[i_l, j_l] f_p[k']) / H_l[i_l, j_l]
//   eq. (norm): |C^(l)|^2 += 2 Re sum_p <H_l, H_p><f_l, f_p> + |H_l|^2 |f_l|^2
//   stop when |H_l| |f_l| <= eps |C^(l)|, else k_{l+1} = tie-argmax over unused k of |f_l|.
//
// Mixed precision: faces, residuals and face factors are FP32 (float2) and every face is
// kept divided by the block scale c_k = exp(-s_k d0) (d0 = distance of the cluster
// centres), so neither the e^{-Re(s) r} decay nor the phase Im(s) r leaves the FP32 range;
// the crosses stay exact because the scale moves into the FP64 fibres:
//   C ~ sum_p H~_p (x) f_p,  R~(:,:,k) = E(:,:,k)/c_k - sum_p (f_p[k]/c_k) H~_p.
// Fibres, Gram values, norms, stop tests and pivot comparisons are FP64.
//
// Two variants share the per-cross tail:
//   small blocks (m n <= MNMAX, m, n <= SIDE): the residual face R and its approximation
//     S = sum_q u_q w_q^T live in LDS and are updated in place by rank-1 updates, so the
//     ACA steps never re-read the factor history; |S|_F^2 is summed directly and
//     H_l = S needs no separate expansion;
//   large blocks: R, H_l and the factor history in HBM scratch (L2 resident), row and
//     column corrections split over thread groups with pipelined loads.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "entries_dev.h"
#include "galerkin_dev.h"
#include "kernels.h"

namespace gaca {

constexpr int kMaxRowsLds = 8192;
constexpr int kMaxLds = 1024;
constexpr int kMaxRcap = 256;
constexpr int kMaxRcapSmall = 64;

// Face entry at (il, jl, kk): FP64 value (FT = double2), the dense test tensor, or the
// scaled FP32 value (FT = float2).
template <int KERNEL, bool DENSE, class FT>
__device__ __forceinline__ FT face_entry(const GeoDev &g, const FreqDev &f, const FarLaunch &fl,
                                         const FarBlockDev &B, int il, int jl, int kk) {
    if (DENSE) return from_d2<FT>(fl.dense[((int64_t)il * B.n + jl) * f.L + kk]);
    const int64_t gi = B.r0 + il, gj = B.c0 + jl;
    if constexpr (KERNEL == 2) {
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
                                               const FarLaunch &fl, const FarBlockDev &B,
                                               int il, int jl, int kk) {
    if (DENSE) return fl.dense[((int64_t)il * B.n + jl) * f.L + kk];
    const int64_t gi = B.r0 + il, gj = B.c0 + jl;
    double er, ei;
    if constexpr (KERNEL == 2)
        entry_gal36(g, gi, gj, f.re[kk], f.im[kk], er, ei);
    else
        entry_far6<KERNEL>(g, g.xx[gi], g.xy[gi], g.xz[gi], gj, f.re[kk], f.im[kk], er, ei);
    return make_double2(er, ei);
}

// 1 / c_k = exp(s_k d0) (mixed scaling), FP64.
__device__ __forceinline__ double2 inv_scale(const FreqDev &f, const FarBlockDev &B, int k) {
    const double d0 = (double)B.d0f;
    const double mag = exp(f.re[k] * d0);
    double sn, cs;
    sincos(f.im[k] * d0, &sn, &cs);
    return make_double2(mag * cs, mag * sn);
}

struct FarState {
    int ell = 0, k = 0, zero_run = 0, zero_faces = 0, capped = 0, sum_rho = 0, nused_k = 0;
    double norm2 = 0.0, scale = 0.0;
};

// Residual face into dst (LDS or HBM); returns ||C^(l-1)(:,:,k)||^2 in the face's frame
// and writes the face's zero threshold factor (1 or 1/|c_k|) to *zscale.
template <int KERNEL, int NT, bool DENSE, bool MIXED, class FT>
__device__ double residual_face(const GeoDev &g, const FreqDev &f, const FarLaunch &fl,
                                const FarBlockDev &B, const FarState &S, const FT *faces,
                                const double2 *fib, const double2 *G, int rcap,
                                double2 *coefd, FT *dst, FT *zero_dst, double *zscale,
                                Red<NT> &red) {
    const int tid = threadIdx.x, L = f.L, n = B.n;
    const int64_t mn = (int64_t)B.m * n;
    double2 isc = make_double2(1.0, 0.0);
    if (MIXED) isc = inv_scale(f, B, S.k);
    for (int p = tid; p < S.ell; p += NT) {
        coefd[p] = cmul(fib[(int64_t)p * L + S.k], isc);
    }
    *zscale = MIXED ? sqrt(cabs2(isc)) : 1.0;
    __syncthreads();
    for (int64_t idx = tid; idx < mn; idx += NT) {
        const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
        FT e = face_entry<KERNEL, DENSE, FT>(g, f, fl, B, i, j, S.k);
        for (int p = 0; p < S.ell; ++p)
            e = csub(e, cmul(from_d2<FT>(coefd[p]), faces[(int64_t)p * mn + idx]));
        dst[idx] = e;
        if (zero_dst) zero_dst[idx] = czero<FT>();
    }
    double part = 0.0;
    for (int a = tid; a < S.ell; a += NT)
        for (int b = 0; b < S.ell; ++b)
            part += cmul(cmulc(coefd[a], coefd[b]), G[(int64_t)a * rcap + b]).x;
    return fmax(red.sum(part), 0.0);
}

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
__device__ int first_unused(const unsigned char *used, int len, Red<NT> &red) {
    int c = len;
    for (int t = threadIdx.x; t < len; t += NT)
        if (!used[t]) {
            c = t;
            break;
        }
    return red.imin(c);
}

// Everything after the face ACA, given H_l at Hl (LDS or HBM) and its copy in the HBM slot
// of face l: pivot, Gram, fibre, eq. (norm), output, stop test, next frequency.
// Returns true when the block is finished.
template <int KERNEL, int NT, bool DENSE, bool MIXED, class FT>
__device__ bool far_cross_tail(const GeoDev &g, const FreqDev &f, const AcaParams &P,
                               const FarLaunch &fl, const FarBlockDev &B, FarState &S,
                               FT *faces, const FT *Ub, const FT *Wb, double2 *fib, double2 *G,
                               const FT *Hl, int rho, double mxh, double h2,
                               unsigned char *used_k, Red<NT> &red, unsigned long long *sh_off) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int NW = NT / 64;
    const int m = B.m, n = B.n, L = f.L, rcap = P.rcap;
    const int64_t mn = (int64_t)m * n;
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);
    const int ell = S.ell;
    // pivot: lowest row-major index with |H|^2 >= (1 - tie)^2 max |H|^2
    const double thh = tie2 * mxh;
    int pc = 0x7fffffff;
    for (int64_t idx = tid; idx < mn; idx += NT)
        if (cabs2(Hl[idx]) >= thh) {
            pc = (int)idx;
            break;
        }
    const int pidx = red.imin(pc);
    const double2 hpiv = to_d2(Hl[pidx]);
    const int ip = pidx / n, jpv = pidx - ip * n;
    // Gram <H_l, H_p>, p < l, accumulated in FP64: four p per wave iteration
    for (int p0 = wave * 4; p0 < ell; p0 += NW * 4) {
        double gr[4] = {0, 0, 0, 0}, gi[4] = {0, 0, 0, 0};
        const int np = min(4, ell - p0);
        for (int64_t idx = lane; idx < mn; idx += 64) {
            const double2 h = to_d2(Hl[idx]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < np) {
                    double2 v = cmulc(h, to_d2(faces[(int64_t)(p0 + t) * mn + idx]));
                    gr[t] += v.x;
                    gi[t] += v.y;
                }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            gr[t] = wave_sum(gr[t]);
            gi[t] = wave_sum(gi[t]);
        }
        if (lane == 0)
            for (int t = 0; t < np; ++t) {
                G[(int64_t)ell * rcap + p0 + t] = make_double2(gr[t], gi[t]);
                G[(int64_t)(p0 + t) * rcap + ell] = make_double2(gr[t], -gi[t]);
            }
    }
    if (tid == 0) G[(int64_t)ell * rcap + ell] = make_double2(h2, 0.0);
    // frequency fibre through the pivot (FP64)
    for (int kk = tid; kk < L; kk += NT) {
        double2 e = fibre_entry<KERNEL, DENSE>(g, f, fl, B, ip, jpv, kk);
        for (int p = 0; p < ell; ++p)
            e = csub(e, cmul(to_d2(faces[(int64_t)p * mn + pidx]), fib[(int64_t)p * L + kk]));
        fib[(int64_t)ell * L + kk] = cdiv(e, hpiv);
    }
    __syncthreads();
    // eq. (norm) update
    const double2 *fl_ = fib + (int64_t)ell * L;
    double c3 = 0.0, f2 = 0.0, fmx = 0.0;
    for (int p = wave; p < ell; p += NW) {
        double dr = 0.0, di = 0.0;
        for (int kk = lane; kk < L; kk += 64) {
            double2 t = cmulc(fl_[kk], fib[(int64_t)p * L + kk]);
            dr += t.x;
            di += t.y;
        }
        dr = wave_sum(dr);
        di = wave_sum(di);
        double2 gv = G[(int64_t)ell * rcap + p];
        c3 += gv.x * dr - gv.y * di;
    }
    if (lane != 0) c3 = 0.0;
    for (int kk = tid; kk < L; kk += NT) {
        double a2 = cabs2(fl_[kk]);
        f2 += a2;
        fmx = fmax(fmx, a2);
    }
    fmx = red.max(fmx);
    double unused0 = 0.0;
    red.sum3(c3, f2, unused0);
    S.norm2 = S.norm2 + 2.0 * c3 + h2 * f2;
    S.scale = fmax(S.scale, sqrt(cabs2(hpiv)) * sqrt(fmx));
    // output: this cross's factors to the arena
    const int64_t nfac = (int64_t)rho * (m + n);
    if (tid == 0) {
        *sh_off = atomicAdd(fl.arena_ctr, (unsigned long long)nfac);
        fl.cmeta[(int64_t)B.out_idx * rcap + ell] = CrossMeta{S.k, ip, jpv, rho};
    }
    __syncthreads();
    const unsigned long long off = *sh_off;
    FT *arena = reinterpret_cast<FT *>(fl.arena);
    if (off + nfac <= fl.arena_cap) {
        for (int64_t t = tid; t < (int64_t)rho * m; t += NT) arena[off + t] = Ub[t];
        for (int64_t t = tid; t < (int64_t)rho * n; t += NT) arena[off + (int64_t)rho * m + t] = Wb[t];
        if (tid == 0) fl.cross_off[(int64_t)B.out_idx * rcap + ell] = (int64_t)off;
    } else if (tid == 0) {
        *fl.overflow = 1;
        fl.cross_off[(int64_t)B.out_idx * rcap + ell] = -1;
    }
    S.sum_rho += rho;
    S.ell = ell + 1;
    if (sqrt(h2 * f2) <= P.eps * sqrt(fmax(S.norm2, 0.0))) return true;
    if (S.nused_k >= L) return true;
    if (S.ell >= rcap) {
        S.capped = 1;
        return true;
    }
    S.k = tie_argmax_unused<NT>(fl_, used_k, L, tie2, red);
    return false;
}

// Zero face bookkeeping; returns true when the block is finished.
template <int NT>
__device__ bool zero_face(FarState &S, const unsigned char *used_k, int L, Red<NT> &red) {
    ++S.zero_faces;
    ++S.zero_run;
    if (S.zero_run >= 3 || S.nused_k >= L) return true;
    S.k = first_unused<NT>(used_k, L, red);
    return false;
}

template <int NT>
__device__ void far_finalize(const FarLaunch &fl, const FarBlockDev &B, const FarState &S,
                             const double2 *fib, int L, unsigned long long *sh_off) {
    const int tid = threadIdx.x;
    const int64_t nf = (int64_t)S.ell * L;
    if (tid == 0) *sh_off = nf > 0 ? atomicAdd(fl.fib_ctr, (unsigned long long)nf) : 0ull;
    __syncthreads();
    const unsigned long long foff = *sh_off;
    if (foff + nf <= fl.fib_cap) {
        for (int64_t t = tid; t < nf; t += NT) fl.fib_arena[foff + t] = fib[t];
        if (tid == 0) fl.fib_off[B.out_idx] = (int64_t)foff;
    } else if (tid == 0) {
        *fl.overflow = 1;
        fl.fib_off[B.out_idx] = -1;
    }
    if (tid == 0) {
        FarMeta mt;
        mt.rank = S.ell;
        mt.sum_rho = S.sum_rho;
        mt.capped = S.capped;
        mt.zero_faces = S.zero_faces;
        mt.fac_off = 0;
        mt.norm2 = S.norm2;
        fl.meta[B.out_idx] = mt;
    }
}

template <class FT>
struct Scratch {
    FT *faces, *Ub, *Wb;
    double2 *fib, *G;
    __device__ Scratch(const FarLaunch &fl, const FarBlockDev &B) {
        char *base = reinterpret_cast<char *>(fl.scratch);
        faces = reinterpret_cast<FT *>(base + B.face_off);
        Ub = reinterpret_cast<FT *>(base + B.uw_off);
        Wb = Ub + (int64_t)B.rho_max * B.m;
        fib = reinterpret_cast<double2 *>(base + B.fib_off);
        G = reinterpret_cast<double2 *>(base + B.gram_off);
    }
};

// ---------------------------------------------------------------------------------------
// Small blocks: R and S in LDS.
template <int KERNEL, int NT, bool DENSE, bool MIXED, int MNMAX, int SIDE>
__global__ void __launch_bounds__(NT)
    far_small_kernel(GeoDev g, FreqDev f, AcaParams P, FarLaunch fl) {
    using FT = typename std::conditional<MIXED, float2, double2>::type;
    const FarBlockDev B = fl.blocks[blockIdx.x];
    const int m = B.m, n = B.n, L = f.L;
    const int mn = m * n;
    const int tid = threadIdx.x;
    Scratch<FT> sc(fl, B);

    __shared__ FT Rs[MNMAX];
    __shared__ FT Ss[MNMAX];
    __shared__ FT ucol[SIDE];
    __shared__ FT wrow[SIDE];
    __shared__ double2 coefd[kMaxRcapSmall];
    __shared__ unsigned char used_row[SIDE];
    __shared__ unsigned char used_k[kMaxLds];
    __shared__ double redbuf[4 * (NT / 64) + 4];
    __shared__ unsigned long long sh_off;
    Red<NT> red{redbuf};
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);

    for (int kk = tid; kk < L; kk += NT) used_k[kk] = 0;
    FarState S;
    __syncthreads();
    while (true) {
        double zs = 1.0;
        const double ref2 = residual_face<KERNEL, NT, DENSE, MIXED, FT>(
            g, f, fl, B, S, sc.faces, sc.fib, sc.G, P.rcap, coefd, Rs, Ss, &zs, red);
        const double zero_tol = P.delta * S.scale * zs;
        for (int r = tid; r < m; r += NT) used_row[r] = 0;
        __syncthreads();
        int q = 0, i = 0, nused = 0;
        double s2 = 0.0;
        while (true) {
            double mx = 0.0;
            for (int j = tid; j < n; j += NT) mx = fmax(mx, cabs2(Rs[i * n + j]));
            mx = red.max(mx);
            if (tid == 0) used_row[i] = 1;
            ++nused;
            if (sqrt(mx) <= zero_tol) {
                __syncthreads();
                const int cand = first_unused<NT>(used_row, m, red);
                if (cand >= m) break;
                i = cand;
                continue;
            }
            const double thr = tie2 * mx;
            int jc = n;
            for (int j = tid; j < n; j += NT)
                if (cabs2(Rs[i * n + j]) >= thr) {
                    jc = j;
                    break;
                }
            const int jp = red.imin(jc);
            const FT piv = Rs[i * n + jp];
            double nw2 = 0.0, nu2 = 0.0;
            for (int j = tid; j < n; j += NT) {
                const FT w = cdiv(Rs[i * n + j], piv);
                wrow[j] = w;
                sc.Wb[(int64_t)q * n + j] = w;
                nw2 += cabs2(w);
            }
            for (int r = tid; r < m; r += NT) {
                const FT u = Rs[r * n + jp];
                ucol[r] = u;
                sc.Ub[(int64_t)q * m + r] = u;
                nu2 += cabs2(u);
            }
            __syncthreads();
            double sp = 0.0;
            for (int idx = tid; idx < mn; idx += NT) {
                const int r = idx / n, j = idx - r * n;
                const FT t = cmul(ucol[r], wrow[j]);
                Rs[idx] = csub(Rs[idx], t);
                const FT sv = cadd(Ss[idx], t);
                Ss[idx] = sv;
                sp += cabs2(sv);
            }
            red.sum3(nu2, nw2, sp);
            s2 = sp;
            ++q;
            if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max)
                break;
            i = tie_argmax_unused<NT>(ucol, used_row, m, tie2, red);
        }
        const int rho = q;
        if (tid == 0) used_k[S.k] = 1;
        ++S.nused_k;
        __syncthreads();
        if (rho == 0) {
            if (zero_face<NT>(S, used_k, L, red)) break;
            continue;
        }
        S.zero_run = 0;
        // H_l = S: store to its HBM slot (needed by later residual faces)
        FT *Hslot = sc.faces + (int64_t)S.ell * mn;
        double mxh = 0.0, h2 = 0.0;
        for (int idx = tid; idx < mn; idx += NT) {
            const FT h = Ss[idx];
            Hslot[idx] = h;
            const double a2 = cabs2(h);
            mxh = fmax(mxh, a2);
            h2 += a2;
        }
        red.maxsum(mxh, h2);
        if (far_cross_tail<KERNEL, NT, DENSE, MIXED, FT>(g, f, P, fl, B, S, sc.faces, sc.Ub, sc.Wb,
                                                         sc.fib, sc.G, Ss, rho, mxh, h2, used_k,
                                                         red, &sh_off))
            break;
    }
    far_finalize<NT>(fl, B, S, sc.fib, L, &sh_off);
}

// ---------------------------------------------------------------------------------------
// Large blocks: R / H_l and the factor history in HBM scratch.
template <int KERNEL, int NT, bool DENSE, bool MIXED>
__global__ void __launch_bounds__(NT)
    far_large_kernel(GeoDev g, FreqDev f, AcaParams P, FarLaunch fl) {
    using FT = typename std::conditional<MIXED, float2, double2>::type;
    const FarBlockDev B = fl.blocks[blockIdx.x];
    const int m = B.m, n = B.n, L = f.L;
    const int64_t mn = (int64_t)m * n;
    const int tid = threadIdx.x;
    constexpr int NW = NT / 64;
    const int wave = tid >> 6, lane = tid & 63;
    Scratch<FT> sc(fl, B);
    FT *faces = sc.faces, *Ub = sc.Ub, *Wb = sc.Wb;

    __shared__ double2 coefd[kMaxRcap];
    __shared__ FT part[NT];       // split-K partial sums of row / column corrections
    __shared__ unsigned char used_row[kMaxRowsLds];
    __shared__ unsigned char used_k[kMaxLds];
    __shared__ double redbuf[4 * NW + 4];
    __shared__ unsigned long long sh_off;
    Red<NT> red{redbuf};
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);

    for (int kk = tid; kk < L; kk += NT) used_k[kk] = 0;
    FarState S;
    __syncthreads();
    while (true) {
        FT *R = faces + (int64_t)S.ell * mn;
        double zs = 1.0;
        const double ref2 = residual_face<KERNEL, NT, DENSE, MIXED, FT>(
            g, f, fl, B, S, faces, sc.fib, sc.G, P.rcap, coefd, R, (FT *)nullptr, &zs, red);
        const double zero_tol = P.delta * S.scale * zs;
        for (int r = tid; r < m; r += NT) used_row[r] = 0;
        __syncthreads();
        int q = 0, i = 0, nused = 0;
        double s2 = 0.0;
        const int splitw = max(1, NT / n), splitu = max(1, NT / m);
        while (true) {
            FT *Wq = Wb + (int64_t)q * n;
            FT *Uq = Ub + (int64_t)q * m;
            // row i of R - sum_{q'<q} u_q'[i] w_q'
            double mx = 0.0;
            if (splitw > 1) {
                const int s = tid / n, j = tid - s * n;
                if (s < splitw) {
                    const int q0 = (int)((int64_t)q * s / splitw), q1 = (int)((int64_t)q * (s + 1) / splitw);
                    part[tid] = dot_strided<FT>(Ub + i, m, Wb + j, n, q0, q1);
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
                    FT v = csub(R[(int64_t)i * n + j], dot_strided<FT>(Ub + i, m, Wb + j, n, 0, q));
                    Wq[j] = v;
                    mx = fmax(mx, cabs2(v));
                }
            }
            mx = red.max(mx);
            if (tid == 0) used_row[i] = 1;
            ++nused;
            if (sqrt(mx) <= zero_tol) {
                __syncthreads();
                const int cand = first_unused<NT>(used_row, m, red);
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
            const int jp = red.imin(jc);
            const FT piv = Wq[jp];
            __syncthreads();
            double nw2 = 0.0, nu2 = 0.0;
            for (int j = tid; j < n; j += NT) {
                FT w = cdiv(Wq[j], piv);
                Wq[j] = w;
                nw2 += cabs2(w);
            }
            // column jp of R - sum_{q'<q} w_q'[jp] u_q'
            if (splitu > 1) {
                const int s = tid / m, r = tid - s * m;
                if (s < splitu) {
                    const int q0 = (int)((int64_t)q * s / splitu), q1 = (int)((int64_t)q * (s + 1) / splitu);
                    part[tid] = dot_strided<FT>(Wb + jp, n, Ub + r, m, q0, q1);
                }
                __syncthreads();
                if (tid < m) {
                    FT u = R[(int64_t)tid * n + jp];
                    for (int t = 0; t < splitu; ++t) u = csub(u, part[t * m + tid]);
                    Uq[tid] = u;
                    nu2 += cabs2(u);
                }
            } else {
                for (int r = tid; r < m; r += NT) {
                    FT u = csub(R[(int64_t)r * n + jp], dot_strided<FT>(Wb + jp, n, Ub + r, m, 0, q));
                    Uq[r] = u;
                    nu2 += cabs2(u);
                }
            }
            __syncthreads();
            // sum_{q'<q} Re(<u_q, u_q'> <w_q, w_q'>) in FP64: four q' per wave iteration
            double cr = 0.0;
            for (int q0 = wave * 4; q0 < q; q0 += NW * 4) {
                const int nq = min(4, q - q0);
                double ur[4] = {0, 0, 0, 0}, ui[4] = {0, 0, 0, 0}, wr[4] = {0, 0, 0, 0},
                       wi[4] = {0, 0, 0, 0};
                for (int r = lane; r < m; r += 64) {
                    const double2 u = to_d2(Uq[r]);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < nq) {
                            double2 v = cmulc(u, to_d2(Ub[(int64_t)(q0 + t) * m + r]));
                            ur[t] += v.x;
                            ui[t] += v.y;
                        }
                }
                for (int j = lane; j < n; j += 64) {
                    const double2 w = to_d2(Wq[j]);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < nq) {
                            double2 v = cmulc(w, to_d2(Wb[(int64_t)(q0 + t) * n + j]));
                            wr[t] += v.x;
                            wi[t] += v.y;
                        }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    ur[t] = wave_sum(ur[t]);
                    ui[t] = wave_sum(ui[t]);
                    wr[t] = wave_sum(wr[t]);
                    wi[t] = wave_sum(wi[t]);
                    if (t < nq) cr += ur[t] * wr[t] - ui[t] * wi[t];
                }
            }
            if (lane != 0) cr = 0.0;
            red.sum3(nu2, nw2, cr);
            s2 = s2 + 2.0 * cr + nu2 * nw2;
            ++q;
            if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max)
                break;
            i = tie_argmax_unused<NT>(Uq, used_row, m, tie2, red);
        }
        const int rho = q;
        if (tid == 0) used_k[S.k] = 1;
        ++S.nused_k;
        __syncthreads();
        if (rho == 0) {
            if (zero_face<NT>(S, used_k, L, red)) break;
            continue;
        }
        S.zero_run = 0;
        // dense expansion H_l = U W^T into the slot of R
        double mxh = 0.0, h2 = 0.0;
        for (int64_t idx = tid; idx < mn; idx += NT) {
            const int ii = (int)(idx / n), jj = (int)(idx - (int64_t)ii * n);
            const FT h = dot_strided<FT>(Ub + ii, m, Wb + jj, n, 0, rho);
            R[idx] = h;
            const double a2 = cabs2(h);
            mxh = fmax(mxh, a2);
            h2 += a2;
        }
        red.maxsum(mxh, h2);
        if (far_cross_tail<KERNEL, NT, DENSE, MIXED, FT>(g, f, P, fl, B, S, faces, Ub, Wb, sc.fib,
                                                         sc.G, R, rho, mxh, h2, used_k, red,
                                                         &sh_off))
            break;
    }
    far_finalize<NT>(fl, B, S, sc.fib, L, &sh_off);
}

// kind: 0 small-A (m n <= 1024, sides <= 64), 1 small-B (m n <= 2304, sides <= 96),
// 2 large.
template <int K, bool D, bool MX>
static void far_dispatch(const GeoDev &g, const FreqDev &f, const AcaParams &P,
                         const FarLaunch &fl, hipStream_t st) {
    dim3 grid(fl.nb);
    if (fl.kind == 0)
        far_small_kernel<K, 64, D, MX, 1024, 64><<<grid, 64, 0, st>>>(g, f, P, fl);
    else if (fl.kind == 1)
        far_small_kernel<K, 256, D, MX, 2304, 96><<<grid, 256, 0, st>>>(g, f, P, fl);
    else
        far_large_kernel<K, 512, D, MX><<<grid, 512, 0, st>>>(g, f, P, fl);
}

void launch_far(int kernel, const GeoDev &g, const FreqDev &f, const AcaParams &P,
                const FarLaunch &fl, hipStream_t st) {
    if (fl.nb <= 0) return;
    if (fl.dense) far_dispatch<0, true, false>(g, f, P, fl, st);
    else if (!fl.mixed) {
        if (kernel == 0) far_dispatch<0, false, false>(g, f, P, fl, st);
        else if (kernel == 1) far_dispatch<1, false, false>(g, f, P, fl, st);
        else far_dispatch<2, false, false>(g, f, P, fl, st);
    } else {
        if (kernel == 0) far_dispatch<0, false, true>(g, f, P, fl, st);
        else if (kernel == 1) far_dispatch<1, false, true>(g, f, P, fl, st);
        else far_dispatch<2, false, true>(g, f, P, fl, st);
    }
}

}  // namespace gaca
