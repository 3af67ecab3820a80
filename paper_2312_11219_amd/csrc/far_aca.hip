// FP64 3D-ACA of far (admissible) blocks, Algorithm 1 of the paper with ACA faces and the
// dense-expansion pivot, one workgroup per block.
//
// Per face l (frequency k_l):
//   residual face R = ENTRY(:, :, k) - sum_{p < l} f_p[k] H_p   (previous dense faces H_p)
//   partial-pivot ACA of R  -> u_q, w_q, stop when |u||w| <= eps_aca sqrt(|C(:,:,k)|^2 + |S|^2)
//   H_l = sum_q u_q w_q^T, pivot (i_l, j_l) = tie-argmax |H_l|
//   fibre f_l[k'] = (ENTRY(i_l, j_l, k') - sum_p H_p[i_l, j_l] f_p[k']) / H_l[i_l, j_l]
//   eq. (norm): |C^(l)|^2 += 2 Re sum_p <H_l, H_p><f_l, f_p> + |H_l|^2 |f_l|^2
//   stop when |H_l| |f_l| <= eps |C^(l)|, else k_{l+1} = tie-argmax over unused k of |f_l|.
//
// Two variants share the per-cross tail:
//   small blocks (m n <= MNMAX, m, n <= SIDE): the residual face R and its approximation
//     S = sum_q u_q w_q^T live in LDS and are updated in place by rank-1 updates, so the
//     ACA steps never re-read the factor history; |S|_F^2 is summed directly and
//     H_l = S needs no separate expansion;
//   large blocks: R, H_l and the factor history in HBM scratch (L2 resident), row and
//     column corrections split over thread groups with pipelined loads.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "entries_dev.h"
#include "kernels.h"

namespace gaca {

constexpr int kMaxRowsLds = 8192;
constexpr int kMaxLds = 1024;
constexpr int kMaxRcap = 256;
constexpr int kMaxRcapSmall = 64;

template <int KERNEL, bool DENSE>
__device__ __forceinline__ double2 far_entry(const GeoDev &g, const FreqDev &f,
                                             const FarLaunch &fl, const FarBlockDev &B, int il,
                                             int jl, int kk) {
    if (DENSE) return fl.dense[((int64_t)il * B.n + jl) * f.L + kk];
    const int64_t gi = B.r0 + il, gj = B.c0 + jl;
    double er, ei;
    entry_far6<KERNEL>(g, g.xx[gi], g.xy[gi], g.xz[gi], gj, f.re[kk], f.im[kk], er, ei);
    return make_double2(er, ei);
}

struct FarState {
    int ell = 0, k = 0, zero_run = 0, zero_faces = 0, capped = 0, sum_rho = 0, nused_k = 0;
    double norm2 = 0.0, scale = 0.0;
};

// Residual face into dst (LDS or HBM) and ||C^(l-1)(:,:,k)||^2.
template <int KERNEL, int NT, bool DENSE>
__device__ double residual_face(const GeoDev &g, const FreqDev &f, const FarLaunch &fl,
                                const FarBlockDev &B, const FarState &S, const double2 *faces,
                                const double2 *fib, const double2 *G, int rcap, double2 *coef,
                                double2 *dst, double2 *zero_dst, Red<NT> &red) {
    const int tid = threadIdx.x, L = f.L, n = B.n;
    const int64_t mn = (int64_t)B.m * n;
    for (int p = tid; p < S.ell; p += NT) coef[p] = fib[(int64_t)p * L + S.k];
    __syncthreads();
    for (int64_t idx = tid; idx < mn; idx += NT) {
        const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
        double2 e = far_entry<KERNEL, DENSE>(g, f, fl, B, i, j, S.k);
        for (int p = 0; p < S.ell; ++p) e = csub(e, cmul(coef[p], faces[(int64_t)p * mn + idx]));
        dst[idx] = e;
        if (zero_dst) zero_dst[idx] = make_double2(0.0, 0.0);
    }
    double part = 0.0;
    for (int a = tid; a < S.ell; a += NT)
        for (int b = 0; b < S.ell; ++b)
            part += cmul(cmulc(coef[a], coef[b]), G[(int64_t)a * rcap + b]).x;
    return fmax(red.sum(part), 0.0);
}

// Tie-argmax helpers over a contiguous array (LDS or HBM), optionally masked.
template <int NT>
__device__ int tie_argmax(const double2 *v, int len, double tie2, Red<NT> &red) {
    double mx = 0.0;
    for (int t = threadIdx.x; t < len; t += NT) mx = fmax(mx, cabs2(v[t]));
    mx = red.max(mx);
    const double thr = tie2 * mx;
    int c = 0x7fffffff;
    for (int t = threadIdx.x; t < len; t += NT)
        if (cabs2(v[t]) >= thr) {
            c = t;
            break;
        }
    return red.imin(c);
}

template <int NT>
__device__ int tie_argmax_unused(const double2 *v, const unsigned char *used, int len,
                                 double tie2, Red<NT> &red) {
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

// Everything after the face ACA: H_l (at Hl, any address space; it is also copied to the
// HBM slot `slot` when Hl is in LDS) -> pivot, Gram, fibre, eq. (norm), output, stop test,
// next frequency.  Returns true when the block is finished.
template <int KERNEL, int NT, bool DENSE>
__device__ bool far_cross_tail(const GeoDev &g, const FreqDev &f, const AcaParams &P,
                               const FarLaunch &fl, const FarBlockDev &B, FarState &S,
                               double2 *faces, const double2 *Ub, const double2 *Wb,
                               double2 *fib, double2 *G, const double2 *Hl, int rho,
                               double mxh, double h2, unsigned char *used_k, Red<NT> &red,
                               unsigned long long *sh_off) {
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
    const double2 hpiv = Hl[pidx];
    const int ip = pidx / n, jpv = pidx - ip * n;
    // Gram <H_l, H_p>, p < l: four p per wave iteration so their loads overlap
    for (int p0 = wave * 4; p0 < ell; p0 += NW * 4) {
        double gr[4] = {0, 0, 0, 0}, gi[4] = {0, 0, 0, 0};
        const int np = min(4, ell - p0);
        for (int64_t idx = lane; idx < mn; idx += 64) {
            const double2 h = Hl[idx];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < np) {
                    double2 v = cmulc(h, faces[(int64_t)(p0 + t) * mn + idx]);
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
    // frequency fibre through the pivot
    for (int kk = tid; kk < L; kk += NT) {
        double2 e = far_entry<KERNEL, DENSE>(g, f, fl, B, ip, jpv, kk);
        for (int p = 0; p < ell; ++p)
            e = csub(e, cmul(faces[(int64_t)p * mn + pidx], fib[(int64_t)p * L + kk]));
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
    if (off + nfac <= fl.arena_cap) {
        for (int64_t t = tid; t < (int64_t)rho * m; t += NT) fl.arena[off + t] = Ub[t];
        for (int64_t t = tid; t < (int64_t)rho * n; t += NT)
            fl.arena[off + (int64_t)rho * m + t] = Wb[t];
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

// ---------------------------------------------------------------------------------------
// Small blocks: R and S in LDS.
template <int KERNEL, int NT, bool DENSE, int MNMAX, int SIDE>
__global__ void __launch_bounds__(NT)
    far_small_kernel(GeoDev g, FreqDev f, AcaParams P, FarLaunch fl) {
    const FarBlockDev B = fl.blocks[blockIdx.x];
    const int m = B.m, n = B.n, L = f.L;
    const int mn = m * n;
    const int tid = threadIdx.x;
    double2 *faces = fl.scratch + B.face_off;
    double2 *Ub = fl.scratch + B.uw_off;
    double2 *Wb = Ub + (int64_t)B.rho_max * m;
    double2 *fib = fl.scratch + B.fib_off;
    double2 *G = fl.scratch + B.gram_off;

    __shared__ double2 Rs[MNMAX];
    __shared__ double2 Ss[MNMAX];
    __shared__ double2 ucol[SIDE];
    __shared__ double2 wrow[SIDE];
    __shared__ double2 coef[kMaxRcapSmall];
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
        const double ref2 = residual_face<KERNEL, NT, DENSE>(g, f, fl, B, S, faces, fib, G, P.rcap,
                                                             coef, Rs, Ss, red);
        const double zero_tol = P.delta * S.scale;
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
            const double2 piv = Rs[i * n + jp];
            double nw2 = 0.0, nu2 = 0.0;
            for (int j = tid; j < n; j += NT) {
                const double2 w = cdiv(Rs[i * n + j], piv);
                wrow[j] = w;
                Wb[(int64_t)q * n + j] = w;
                nw2 += cabs2(w);
            }
            for (int r = tid; r < m; r += NT) {
                const double2 u = Rs[r * n + jp];
                ucol[r] = u;
                Ub[(int64_t)q * m + r] = u;
                nu2 += cabs2(u);
            }
            __syncthreads();
            double sp = 0.0;
            for (int idx = tid; idx < mn; idx += NT) {
                const int r = idx / n, j = idx - r * n;
                const double2 t = cmul(ucol[r], wrow[j]);
                Rs[idx] = csub(Rs[idx], t);
                const double2 sv = cadd(Ss[idx], t);
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
        double2 *Hslot = faces + (int64_t)S.ell * mn;
        double mxh = 0.0, h2 = 0.0;
        for (int idx = tid; idx < mn; idx += NT) {
            const double2 h = Ss[idx];
            Hslot[idx] = h;
            const double a2 = cabs2(h);
            mxh = fmax(mxh, a2);
            h2 += a2;
        }
        red.maxsum(mxh, h2);
        if (far_cross_tail<KERNEL, NT, DENSE>(g, f, P, fl, B, S, faces, Ub, Wb, fib, G, Ss, rho,
                                              mxh, h2, used_k, red, &sh_off))
            break;
    }
    far_finalize<NT>(fl, B, S, fib, L, &sh_off);
}

// ---------------------------------------------------------------------------------------
// Large blocks: R / H_l and the factor history in HBM scratch.
template <int KERNEL, int NT, bool DENSE>
__global__ void __launch_bounds__(NT)
    far_large_kernel(GeoDev g, FreqDev f, AcaParams P, FarLaunch fl) {
    const FarBlockDev B = fl.blocks[blockIdx.x];
    const int m = B.m, n = B.n, L = f.L;
    const int64_t mn = (int64_t)m * n;
    const int tid = threadIdx.x;
    constexpr int NW = NT / 64;
    const int wave = tid >> 6, lane = tid & 63;
    double2 *faces = fl.scratch + B.face_off;
    double2 *Ub = fl.scratch + B.uw_off;
    double2 *Wb = Ub + (int64_t)B.rho_max * m;
    double2 *fib = fl.scratch + B.fib_off;
    double2 *G = fl.scratch + B.gram_off;

    __shared__ double2 coef[kMaxRcap];
    __shared__ double2 part[NT];       // split-K partial sums of row / column corrections
    __shared__ unsigned char used_row[kMaxRowsLds];
    __shared__ unsigned char used_k[kMaxLds];
    __shared__ double redbuf[4 * NW + 4];
    __shared__ double wpart[4 * NW];
    __shared__ unsigned long long sh_off;
    Red<NT> red{redbuf};
    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);

    for (int kk = tid; kk < L; kk += NT) used_k[kk] = 0;
    FarState S;
    __syncthreads();
    while (true) {
        double2 *R = faces + (int64_t)S.ell * mn;
        const double ref2 = residual_face<KERNEL, NT, DENSE>(g, f, fl, B, S, faces, fib, G, P.rcap,
                                                             coef, R, nullptr, red);
        const double zero_tol = P.delta * S.scale;
        for (int r = tid; r < m; r += NT) used_row[r] = 0;
        __syncthreads();
        int q = 0, i = 0, nused = 0;
        double s2 = 0.0;
        // split-K factors: nsplit thread groups per element when the vector is short
        const int splitw = max(1, NT / n), splitu = max(1, NT / m);
        while (true) {
            double2 *Wq = Wb + (int64_t)q * n;
            double2 *Uq = Ub + (int64_t)q * m;
            // row i of R - sum_{q'<q} u_q'[i] w_q'
            double mx = 0.0;
            if (splitw > 1) {
                const int s = tid / n, j = tid - s * n;
                if (s < splitw) {
                    const int q0 = (int)((int64_t)q * s / splitw), q1 = (int)((int64_t)q * (s + 1) / splitw);
                    part[tid] = dot_strided(Ub + i, m, Wb + j, n, q0, q1);
                }
                __syncthreads();
                if (tid < n) {
                    double2 v = R[(int64_t)i * n + tid];
                    for (int t = 0; t < splitw; ++t) v = csub(v, part[t * n + tid]);
                    Wq[tid] = v;
                    mx = cabs2(v);
                }
            } else {
                for (int j = tid; j < n; j += NT) {
                    double2 v = csub(R[(int64_t)i * n + j], dot_strided(Ub + i, m, Wb + j, n, 0, q));
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
            const double2 piv = Wq[jp];
            __syncthreads();
            double nw2 = 0.0, nu2 = 0.0;
            for (int j = tid; j < n; j += NT) {
                double2 w = cdiv(Wq[j], piv);
                Wq[j] = w;
                nw2 += cabs2(w);
            }
            // column jp of R - sum_{q'<q} w_q'[jp] u_q'
            if (splitu > 1) {
                const int s = tid / m, r = tid - s * m;
                if (s < splitu) {
                    const int q0 = (int)((int64_t)q * s / splitu), q1 = (int)((int64_t)q * (s + 1) / splitu);
                    part[tid] = dot_strided(Wb + jp, n, Ub + r, m, q0, q1);
                }
                __syncthreads();
                if (tid < m) {
                    double2 u = R[(int64_t)tid * n + jp];
                    for (int t = 0; t < splitu; ++t) u = csub(u, part[t * m + tid]);
                    Uq[tid] = u;
                    nu2 += cabs2(u);
                }
            } else {
                for (int r = tid; r < m; r += NT) {
                    double2 u = csub(R[(int64_t)r * n + jp], dot_strided(Wb + jp, n, Ub + r, m, 0, q));
                    Uq[r] = u;
                    nu2 += cabs2(u);
                }
            }
            __syncthreads();
            // sum_{q'<q} Re(<u_q, u_q'> <w_q, w_q'>): four q' per wave iteration
            double cr = 0.0;
            for (int q0 = wave * 4; q0 < q; q0 += NW * 4) {
                const int nq = min(4, q - q0);
                double ur[4] = {0, 0, 0, 0}, ui[4] = {0, 0, 0, 0}, wr[4] = {0, 0, 0, 0},
                       wi[4] = {0, 0, 0, 0};
                for (int r = lane; r < m; r += 64) {
                    const double2 u = Uq[r];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < nq) {
                            double2 v = cmulc(u, Ub[(int64_t)(q0 + t) * m + r]);
                            ur[t] += v.x;
                            ui[t] += v.y;
                        }
                }
                for (int j = lane; j < n; j += 64) {
                    const double2 w = Wq[j];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < nq) {
                            double2 v = cmulc(w, Wb[(int64_t)(q0 + t) * n + j]);
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
            const double2 h = dot_strided(Ub + ii, m, Wb + jj, n, 0, rho);
            R[idx] = h;
            const double a2 = cabs2(h);
            mxh = fmax(mxh, a2);
            h2 += a2;
        }
        red.maxsum(mxh, h2);
        if (far_cross_tail<KERNEL, NT, DENSE>(g, f, P, fl, B, S, faces, Ub, Wb, fib, G, R, rho,
                                              mxh, h2, used_k, red, &sh_off))
            break;
    }
    far_finalize<NT>(fl, B, S, fib, L, &sh_off);
}

// kind: 0 small-A (m n <= 1024, sides <= 64), 1 small-B (m n <= 2304, sides <= 96),
// 2 large.
void launch_far_fp64(int kernel, const GeoDev &g, const FreqDev &f, const AcaParams &P,
                     const FarLaunch &fl, hipStream_t st) {
    if (fl.nb <= 0) return;
    dim3 grid(fl.nb);
#define GACA_SMALLA(K, D) far_small_kernel<K, 64, D, 1024, 64><<<grid, 64, 0, st>>>(g, f, P, fl)
#define GACA_SMALLB(K, D) far_small_kernel<K, 256, D, 2304, 96><<<grid, 256, 0, st>>>(g, f, P, fl)
#define GACA_LARGE(K, D) far_large_kernel<K, 512, D><<<grid, 512, 0, st>>>(g, f, P, fl)
#define GACA_KIND(K, D)                        \
    do {                                       \
        if (fl.kind == 0) GACA_SMALLA(K, D);   \
        else if (fl.kind == 1) GACA_SMALLB(K, D); \
        else GACA_LARGE(K, D);                 \
    } while (0)
    if (fl.dense) GACA_KIND(0, true);
    else if (kernel == 0) GACA_KIND(0, false);
    else GACA_KIND(1, false);
#undef GACA_KIND
#undef GACA_LARGE
#undef GACA_SMALLB
#undef GACA_SMALLA
}

}  // namespace gaca
