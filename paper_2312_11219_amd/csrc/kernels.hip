// HIP kernels of libgaca for gfx950 (MI355X): dense near field, FP64 3D-ACA of far
// blocks (Algorithm 1 with ACA faces and the dense-expansion pivot), entry test hook and
// the FP64 reordered product eq. (product).
#include <hip/hip_runtime.h>

#include "entries_dev.h"
#include "kernels.h"

namespace gaca {

// ---------------------------------------------------------------------------------------
// small complex helpers (double2 = (re, im))
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------------------------------
// wave64 / workgroup reductions (fixed order: deterministic)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

template <int NT>
struct Red {
    static constexpr int NW = NT / 64;
    double *buf;   // >= 4 * NW doubles of shared memory
    __device__ double sum(double v) {
        v = wave_sum(v);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += buf[w];
        return t;
    }
    __device__ void sum3(double &a, double &b, double &c) {
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            buf[3 * (threadIdx.x >> 6)] = a;
            buf[3 * (threadIdx.x >> 6) + 1] = b;
            buf[3 * (threadIdx.x >> 6) + 2] = c;
        }
        __syncthreads();
        a = b = c = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            a += buf[3 * w];
            b += buf[3 * w + 1];
            c += buf[3 * w + 2];
        }
    }
    __device__ double max(double v) {
        v = wave_max(v);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = buf[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) t = fmax(t, buf[w]);
        return t;
    }
    __device__ int imin(int v) {
        v = wave_min(v);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) reinterpret_cast<int *>(buf)[threadIdx.x >> 6] = v;
        __syncthreads();
        int t = reinterpret_cast<int *>(buf)[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) t = min(t, reinterpret_cast<int *>(buf)[w]);
        return t;
    }
};

// ---------------------------------------------------------------------------------------
// Near field: one thread per (pair, chunk of NF frequencies) of one quadrature tier.
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

void launch_near(int kernel, int tier, const GeoDev &g, const QuadDev &q, const FreqDev &f,
                 const NearPair *pairs, int64_t npairs, const NearBlockDev *blocks,
                 double2 *out64, float2 *out32, hipStream_t st) {
    if (npairs <= 0) return;
    constexpr int NF = 8;
    dim3 grid((unsigned)((npairs + 255) / 256), (unsigned)((f.L_eval + NF - 1) / NF));
#define GACA_NEAR(K, T) \
    near_kernel<K, T, NF><<<grid, 256, 0, st>>>(g, q, f, pairs, npairs, blocks, out64, out32)
    if (kernel == 0) {
        switch (tier) {
            case TIER_FAR6: GACA_NEAR(0, TIER_FAR6); break;
            case TIER_MID4: GACA_NEAR(0, TIER_MID4); break;
            case TIER_NEAR8: GACA_NEAR(0, TIER_NEAR8); break;
            default: GACA_NEAR(0, TIER_SELF); break;
        }
    } else {
        switch (tier) {
            case TIER_FAR6: GACA_NEAR(1, TIER_FAR6); break;
            case TIER_MID4: GACA_NEAR(1, TIER_MID4); break;
            case TIER_NEAR8: GACA_NEAR(1, TIER_NEAR8); break;
            default: GACA_NEAR(1, TIER_SELF); break;
        }
    }
#undef GACA_NEAR
}

// ---------------------------------------------------------------------------------------
// Entry test hook
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
    else
        eval_kernel<1><<<nb, 128, 0, st>>>(g, q, f, n, rows, cols, ks, tiers, out);
}

// ---------------------------------------------------------------------------------------
// FP64 3D-ACA of one far block per workgroup (Algorithm 1).
//
// Scratch per block (HBM, L2-resident for small blocks):
//   faces[rcap][m*n]  dense faces H_p = U_p W_p^T; slot l first holds the residual face
//   U[rho_max][m], W[rho_max][n]  factors of the face being built (column-major)
//   fib[rcap][L]      fibres f_p
//   G[rcap][rcap]     Gram values <H_a, H_b>_F of eq. (norm)
// Every decision (pivots, stop tests) is taken from workgroup reductions that all threads
// see, so the control flow is uniform.
constexpr int kMaxRowsLds = 8192;
constexpr int kMaxLds = 1024;
constexpr int kMaxRcap = 256;

template <int KERNEL, int NT, bool DENSE>
__global__ void __launch_bounds__(NT)
    far_fp64_kernel(GeoDev g, FreqDev f, AcaParams P, FarLaunch fl) {
    const FarBlockDev B = fl.blocks[blockIdx.x];
    const int m = B.m, n = B.n, L = f.L, rcap = P.rcap;
    const int64_t mn = (int64_t)m * n;
    const int tid = threadIdx.x;
    constexpr int NW = NT / 64;
    const int wave = tid >> 6, lane = tid & 63;
    double2 *faces = fl.scratch + B.face_off;
    double2 *Ub = fl.scratch + B.uw_off;
    double2 *Wb = Ub + (int64_t)B.rho_max * m;
    double2 *fib = fl.scratch + B.fib_off;
    double2 *G = fl.scratch + B.gram_off;

    __shared__ double redbuf[4 * NW + 4];
    __shared__ double2 coef[kMaxRcap];
    __shared__ unsigned char used_row[kMaxRowsLds];
    __shared__ unsigned char used_k[kMaxLds];
    __shared__ double wpart[3 * NW];
    __shared__ unsigned long long sh_off;
    Red<NT> red{redbuf};

    const double tie2 = (1.0 - P.tie) * (1.0 - P.tie);
    auto entry = [&](int il, int jl, int kk) -> double2 {
        if (DENSE) return fl.dense[((int64_t)il * n + jl) * L + kk];
        const int64_t gi = B.r0 + il, gj = B.c0 + jl;
        double er, ei;
        entry_far6<KERNEL>(g, g.xx[gi], g.xy[gi], g.xz[gi], gj, f.re[kk], f.im[kk], er, ei);
        return make_double2(er, ei);
    };

    for (int kk = tid; kk < L; kk += NT) used_k[kk] = 0;
    int ell = 0, k = 0, zero_run = 0, zero_faces = 0, capped = 0, sum_rho = 0, nused_k = 0;
    double norm2 = 0.0, scale = 0.0;
    __syncthreads();

    while (true) {
        double2 *R = faces + (int64_t)ell * mn;
        for (int p = tid; p < ell; p += NT) coef[p] = fib[(int64_t)p * L + k];
        __syncthreads();
        // residual face ENTRY(:, :, k) - C^(l-1)(:, :, k)
        for (int64_t idx = tid; idx < mn; idx += NT) {
            const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
            double2 e = entry(i, j, k);
            for (int p = 0; p < ell; ++p) e = csub(e, cmul(coef[p], faces[(int64_t)p * mn + idx]));
            R[idx] = e;
        }
        // ||C^(l-1)(:,:,k)||_F^2 = sum_ab f_a[k] conj(f_b[k]) <H_a, H_b>
        double part = 0.0;
        for (int a = tid; a < ell; a += NT)
            for (int b = 0; b < ell; ++b) {
                double2 t = cmul(cmulc(coef[a], coef[b]), G[(int64_t)a * rcap + b]);
                part += t.x;
            }
        const double ref2 = fmax(red.sum(part), 0.0);
        const double zero_tol = P.delta * scale;
        // ---- face ACA (partial pivoting) on R ----
        for (int r = tid; r < m; r += NT) used_row[r] = 0;
        __syncthreads();
        int q = 0, i = 0, nused = 0;
        double s2 = 0.0;
        while (true) {
            double2 *Wq = Wb + (int64_t)q * n;
            double2 *Uq = Ub + (int64_t)q * m;
            double mx = 0.0;
            for (int j = tid; j < n; j += NT) {
                double2 v = R[(int64_t)i * n + j];
                for (int qq = 0; qq < q; ++qq)
                    v = csub(v, cmul(Ub[(int64_t)qq * m + i], Wb[(int64_t)qq * n + j]));
                Wq[j] = v;
                mx = fmax(mx, cabs2(v));
            }
            mx = red.max(mx);
            if (tid == 0) used_row[i] = 1;
            ++nused;
            if (sqrt(mx) <= zero_tol) {
                __syncthreads();
                int cand = m;
                for (int r = tid; r < m; r += NT)
                    if (!used_row[r]) {
                        cand = r;
                        break;
                    }
                cand = red.imin(cand);
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
            for (int r = tid; r < m; r += NT) {
                double2 u = R[(int64_t)r * n + jp];
                for (int qq = 0; qq < q; ++qq)
                    u = csub(u, cmul(Wb[(int64_t)qq * n + jp], Ub[(int64_t)qq * m + r]));
                Uq[r] = u;
                nu2 += cabs2(u);
            }
            __syncthreads();
            // cross terms sum_{q' < q} Re(<u_q, u_q'> <w_q, w_q'>), one q' per wave at a time
            double cr = 0.0;
            for (int qq = wave; qq < q; qq += NW) {
                double dur = 0.0, dui = 0.0, dwr = 0.0, dwi = 0.0;
                for (int r = lane; r < m; r += 64) {
                    double2 t = cmulc(Uq[r], Ub[(int64_t)qq * m + r]);
                    dur += t.x;
                    dui += t.y;
                }
                for (int j = lane; j < n; j += 64) {
                    double2 t = cmulc(Wq[j], Wb[(int64_t)qq * n + j]);
                    dwr += t.x;
                    dwi += t.y;
                }
                dur = wave_sum(dur);
                dui = wave_sum(dui);
                dwr = wave_sum(dwr);
                dwi = wave_sum(dwi);
                cr += dur * dwr - dui * dwi;
            }
            if (lane != 0) cr = 0.0;
            red.sum3(nu2, nw2, cr);
            s2 = s2 + 2.0 * cr + nu2 * nw2;
            ++q;
            if (sqrt(nu2 * nw2) <= P.eps_aca * sqrt(ref2 + s2) || nused >= m || q >= B.rho_max)
                break;
            // next row: argmax over unused rows of |u|
            double mu = -1.0;
            for (int r = tid; r < m; r += NT)
                if (!used_row[r]) mu = fmax(mu, cabs2(Uq[r]));
            mu = red.max(mu);
            const double thu = tie2 * mu;
            int ic = m;
            for (int r = tid; r < m; r += NT)
                if (!used_row[r] && cabs2(Uq[r]) >= thu) {
                    ic = r;
                    break;
                }
            i = red.imin(ic);
        }
        const int rho = q;
        if (tid == 0) used_k[k] = 1;
        ++nused_k;
        __syncthreads();
        if (rho == 0) {
            ++zero_faces;
            ++zero_run;
            if (zero_run >= 3 || nused_k >= L) break;
            int cand = L;
            for (int kk = tid; kk < L; kk += NT)
                if (!used_k[kk]) {
                    cand = kk;
                    break;
                }
            k = red.imin(cand);
            continue;
        }
        zero_run = 0;
        // ---- dense expansion H_l = U W^T, pivot = tie-argmax |H_l| ----
        double mxh = 0.0, h2 = 0.0;
        for (int64_t idx = tid; idx < mn; idx += NT) {
            const int ii = (int)(idx / n), jj = (int)(idx - (int64_t)ii * n);
            double2 h = make_double2(0.0, 0.0);
            for (int qq = 0; qq < rho; ++qq) {
                double2 t = cmul(Ub[(int64_t)qq * m + ii], Wb[(int64_t)qq * n + jj]);
                h.x += t.x;
                h.y += t.y;
            }
            R[idx] = h;
            const double a2 = cabs2(h);
            mxh = fmax(mxh, a2);
            h2 += a2;
        }
        mxh = red.max(mxh);
        h2 = red.sum(h2);
        const double thh = tie2 * mxh;
        int pc = 0x7fffffff;
        for (int64_t idx = tid; idx < mn; idx += NT)
            if (cabs2(R[idx]) >= thh) {
                pc = (int)idx;
                break;
            }
        const int pidx = red.imin(pc);
        const double2 hpiv = R[pidx];
        const int ip = pidx / n, jpv = pidx - ip * n;
        // ---- Gram <H_l, H_p> for p < l (one p per wave at a time) ----
        for (int p = wave; p < ell; p += NW) {
            double gr = 0.0, gi = 0.0;
            const double2 *Hp = faces + (int64_t)p * mn;
            for (int64_t idx = lane; idx < mn; idx += 64) {
                double2 t = cmulc(R[idx], Hp[idx]);
                gr += t.x;
                gi += t.y;
            }
            gr = wave_sum(gr);
            gi = wave_sum(gi);
            if (lane == 0) {
                G[(int64_t)ell * rcap + p] = make_double2(gr, gi);
                G[(int64_t)p * rcap + ell] = make_double2(gr, -gi);
            }
        }
        if (tid == 0) G[(int64_t)ell * rcap + ell] = make_double2(h2, 0.0);
        // ---- frequency fibre ----
        for (int kk = tid; kk < L; kk += NT) {
            double2 e = entry(ip, jpv, kk);
            for (int p = 0; p < ell; ++p)
                e = csub(e, cmul(faces[(int64_t)p * mn + pidx], fib[(int64_t)p * L + kk]));
            fib[(int64_t)ell * L + kk] = cdiv(e, hpiv);
        }
        __syncthreads();
        // ---- eq. (norm) update ----
        double c3 = 0.0, f2 = 0.0, fmx = 0.0;
        const double2 *fl_ = fib + (int64_t)ell * L;
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
            c3 += gv.x * dr - gv.y * di;   // Re(<H_l,H_p> <f_l,f_p>)
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
        norm2 = norm2 + 2.0 * c3 + h2 * f2;
        scale = fmax(scale, sqrt(cabs2(hpiv)) * sqrt(fmx));
        // ---- store the cross ----
        const int64_t nfac = (int64_t)rho * (m + n);
        if (tid == 0) {
            unsigned long long off = atomicAdd(fl.arena_ctr, (unsigned long long)nfac);
            sh_off = off;
            CrossMeta cm{k, ip, jpv, rho};
            fl.cmeta[(int64_t)B.out_idx * rcap + ell] = cm;
        }
        __syncthreads();
        const unsigned long long off = sh_off;
        if (off + nfac <= fl.arena_cap) {
            for (int64_t t = tid; t < (int64_t)rho * m; t += NT) fl.arena[off + t] = Ub[t];
            for (int64_t t = tid; t < (int64_t)rho * n; t += NT)
                fl.arena[off + (int64_t)rho * m + t] = Wb[t];
            if (tid == 0) fl.cross_off[(int64_t)B.out_idx * rcap + ell] = (int64_t)off;
        } else if (tid == 0) {
            *fl.overflow = 1;
            fl.cross_off[(int64_t)B.out_idx * rcap + ell] = -1;
        }
        sum_rho += rho;
        ++ell;
        if (sqrt(h2 * f2) <= P.eps * sqrt(fmax(norm2, 0.0))) break;
        if (nused_k >= L) break;
        if (ell >= rcap) {
            capped = 1;
            break;
        }
        // ---- next frequency: tie-argmax over unused k of |f_l[k]| ----
        double mf = -1.0;
        for (int kk = tid; kk < L; kk += NT)
            if (!used_k[kk]) mf = fmax(mf, cabs2(fl_[kk]));
        mf = red.max(mf);
        const double thf = tie2 * mf;
        int kc = L;
        for (int kk = tid; kk < L; kk += NT)
            if (!used_k[kk] && cabs2(fl_[kk]) >= thf) {
                kc = kk;
                break;
            }
        k = red.imin(kc);
    }
    // ---- finalize: fibres to their arena, metadata ----
    const int64_t nf = (int64_t)ell * L;
    if (tid == 0) {
        unsigned long long off = nf > 0 ? atomicAdd(fl.fib_ctr, (unsigned long long)nf) : 0ull;
        sh_off = off;
    }
    __syncthreads();
    const unsigned long long foff = sh_off;
    if (foff + nf <= fl.fib_cap) {
        for (int64_t t = tid; t < nf; t += NT) fl.fib_arena[foff + t] = fib[t];
        if (tid == 0) fl.fib_off[B.out_idx] = (int64_t)foff;
    } else if (tid == 0) {
        *fl.overflow = 1;
        fl.fib_off[B.out_idx] = -1;
    }
    if (tid == 0) {
        FarMeta mt;
        mt.rank = ell;
        mt.sum_rho = sum_rho;
        mt.capped = capped;
        mt.zero_faces = zero_faces;
        mt.fac_off = 0;
        mt.norm2 = norm2;
        fl.meta[B.out_idx] = mt;
    }
}

void launch_far_fp64(int kernel, const GeoDev &g, const FreqDev &f, const AcaParams &P,
                     const FarLaunch &fl, hipStream_t st) {
    if (fl.nb <= 0) return;
    dim3 grid(fl.nb);
#define GACA_FAR(K, NT, D) far_fp64_kernel<K, NT, D><<<grid, NT, 0, st>>>(g, f, P, fl)
    if (fl.dense) {
        if (fl.threads == 64) GACA_FAR(0, 64, true);
        else GACA_FAR(0, 256, true);
    } else if (kernel == 0) {
        if (fl.threads == 64) GACA_FAR(0, 64, false);
        else GACA_FAR(0, 256, false);
    } else {
        if (fl.threads == 64) GACA_FAR(1, 64, false);
        else GACA_FAR(1, 256, false);
    }
#undef GACA_FAR
}

// ---------------------------------------------------------------------------------------
// FP64 apply (eq. product), owner-computes per leaf cluster: no atomics, deterministic.
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
