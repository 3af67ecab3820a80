// 3D-ACA of the non-admissible (near-field) blocks with dense faces (Sec. 4 remarks: for
// non-admissible blocks the largest entry is found by comparing all block entries; the
// "No Lwr" variant of Sec. 5: approximation with respect to the frequencies only).
// Algorithm 1 with H_l = the residual face N(:, k_l, :) - sum_{p<l} f_p[k_l] H_p itself:
// pivot = first entry (row-major) with |H_l|^2 >= (1 - tie)^2 max |H_l|^2, fibre through
// it, eq. (norm), stop test, next frequency = argmax over unused |f_l[k]| (tie rule), zero
// faces (max |H_l| <= delta * scale, scale = max_p |H_p[pivot]| max|f_p|): next unused index,
// three in a row or all frequencies used end the block.  One wave (64 lanes) per block, the
// face's entries in registers (up to kNearAcaMaxMN of them), the previous faces and fibres
// in the chunk's scratch (rc slots per block).  FP64 arithmetic; faces stored in the near
// field's storage type.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

namespace {

constexpr int kNE = kNearAcaMaxMN / 64;   // entries per lane

__device__ __forceinline__ double2 cmulq(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <class FT>
__global__ void __launch_bounds__(64) near_aca_kernel(NearAcaArgs q, const FT *near, FT *faces) {
    const int blk = blockIdx.x;            // chunk-local
    const NearBlockDev B = q.blocks[q.b0 + blk];
    const int lane = threadIdx.x;
    const int m = B.m, n = B.n, mn = m * n, L = q.L, rc = q.rc;
    NearAcaOut res{0, 0, 0, 0};
    if (mn > kNearAcaMaxMN) {
        if (lane == 0) {
            res.capped = 1;   // kept dense
            q.out[blk] = res;
        }
        return;
    }
    __shared__ unsigned char used[kNearAcaMaxFreq];
    for (int k = lane; k < L; k += 64) used[k] = 0;
    __syncthreads();
    const FT *N = near + B.off;
    FT *Hs = faces + (int64_t)blk * rc * q.mnmax;          // face p at Hs + p * mnmax
    double2 *Fs = q.fib + (int64_t)blk * rc * L;          // fibre p at Fs + p * L
    const double tie2 = (1.0 - q.tie) * (1.0 - q.tie);
    int k = 0, ell = 0, zero_run = 0, nused = 0, capped = 0, zero_faces = 0;
    double norm2 = 0.0, scale = 0.0;
    double2 R[kNE];
    while (true) {
        // residual face at k
#pragma unroll
        for (int t = 0; t < kNE; ++t) {
            const int e = lane + 64 * t;
            R[t] = make_double2(0.0, 0.0);
            if (e < mn) {
                const int i = e / n, j = e - i * n;
                R[t] = to_d2(N[((int64_t)i * L + k) * n + j]);
            }
        }
        for (int p = 0; p < ell; ++p) {
            const double2 c = Fs[(int64_t)p * L + k];
#pragma unroll
            for (int t = 0; t < kNE; ++t) {
                const int e = lane + 64 * t;
                if (e < mn) {
                    const double2 v = cmulq(c, to_d2(Hs[(int64_t)p * q.mnmax + e]));
                    R[t].x -= v.x;
                    R[t].y -= v.y;
                }
            }
        }
        if (lane == 0) used[k] = 1;
        ++nused;
        double mx = 0.0;
#pragma unroll
        for (int t = 0; t < kNE; ++t) mx = fmax(mx, cabs2(R[t]));
        mx = wave_max(mx);
        __syncthreads();
        if (sqrt(mx) <= q.delta * scale) {
            ++zero_faces;
            ++zero_run;
            if (zero_run >= 3 || nused >= L) break;
            int kk = 0x7fffffff;
            for (int x = lane; x < L; x += 64)
                if (!used[x]) {
                    kk = x;
                    break;
                }
            kk = wave_min(kk);
            k = kk < L ? kk : 0;
            continue;
        }
        zero_run = 0;
        // pivot: lowest entry index at the tie threshold
        int pe = 0x7fffffff;
#pragma unroll
        for (int t = kNE - 1; t >= 0; --t) {   // the lane's lowest qualifying entry wins
            const int e = lane + 64 * t;
            if (e < mn && cabs2(R[t]) >= tie2 * mx) pe = e;
        }
        pe = wave_min(pe);
        if (pe >= mn) pe = 0;   // no entry compares (NaN)
        const int owner = pe & 63, slot = pe >> 6;
        double2 hp = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < kNE; ++t)
            if (t == slot) hp = R[t];
        hp.x = __shfl(hp.x, owner);
        hp.y = __shfl(hp.y, owner);
        // store the face, ||H_l||^2
        double h2 = 0.0;
#pragma unroll
        for (int t = 0; t < kNE; ++t) {
            const int e = lane + 64 * t;
            if (e < mn) {
                Hs[(int64_t)ell * q.mnmax + e] = from_d2<FT>(R[t]);
                h2 += cabs2(R[t]);
            }
        }
        h2 = wave_sum(h2);
        // fibre through the pivot, f[k'] = (N(pe, k') - sum_p H_p(pe) f_p[k']) / H_l(pe)
        const int pi = pe / n, pj = pe - pi * n;
        double2 *fl = Fs + (int64_t)ell * L;
        double f2 = 0.0, fmx = 0.0;
        for (int kk = lane; kk < L; kk += 64) {
            double2 v = to_d2(N[((int64_t)pi * L + kk) * n + pj]);
            for (int p = 0; p < ell; ++p) {
                const double2 w = cmulq(to_d2(Hs[(int64_t)p * q.mnmax + pe]), Fs[(int64_t)p * L + kk]);
                v.x -= w.x;
                v.y -= w.y;
            }
            const double d = hp.x * hp.x + hp.y * hp.y;
            const double2 fv = make_double2((v.x * hp.x + v.y * hp.y) / d, (v.y * hp.x - v.x * hp.y) / d);
            fl[kk] = fv;
            f2 += cabs2(fv);
            fmx = fmax(fmx, cabs2(fv));
        }
        f2 = wave_sum(f2);
        fmx = wave_max(fmx);
        __syncthreads();   // the fibre is read back below by other lanes
        // eq. (norm): 2 Re sum_p <H_l, H_p> <f_p, f_l>
        double c3 = 0.0;
        for (int p = 0; p < ell; ++p) {
            double gr = 0.0, gi = 0.0;
#pragma unroll
            for (int t = 0; t < kNE; ++t) {
                const int e = lane + 64 * t;
                if (e < mn) {
                    const double2 h = to_d2(Hs[(int64_t)p * q.mnmax + e]);
                    gr += R[t].x * h.x + R[t].y * h.y;   // R conj(h)
                    gi += R[t].y * h.x - R[t].x * h.y;
                }
            }
            double dr = 0.0, di = 0.0;
            for (int kk = lane; kk < L; kk += 64) {
                const double2 a = Fs[(int64_t)p * L + kk], b = fl[kk];
                dr += a.x * b.x + a.y * b.y;   // conj(f_p) f_l
                di += a.x * b.y - a.y * b.x;
            }
            gr = wave_sum(gr);
            gi = wave_sum(gi);
            dr = wave_sum(dr);
            di = wave_sum(di);
            c3 += gr * dr - gi * di;
        }
        norm2 = norm2 + 2.0 * c3 + h2 * f2;
        scale = fmax(scale, sqrt(hp.x * hp.x + hp.y * hp.y) * sqrt(fmx));
        ++ell;
        if (sqrt(h2 * f2) <= q.eps * sqrt(fmax(norm2, 0.0))) break;
        if (nused >= L) break;
        if (ell >= rc) {
            capped = 1;
            break;
        }
        // next frequency: argmax over unused |f_l|^2, lowest index at the tie threshold
        double am = 0.0;
        for (int kk = lane; kk < L; kk += 64)
            if (!used[kk]) am = fmax(am, cabs2(fl[kk]));
        am = wave_max(am);
        int kn = 0x7fffffff;
        for (int kk = lane; kk < L; kk += 64)
            if (!used[kk] && cabs2(fl[kk]) >= tie2 * am) {
                kn = kk;
                break;
            }
        kn = wave_min(kn);
        if (kn >= L) {   // no candidate compares (NaN): lowest unused index
            kn = 0x7fffffff;
            for (int kk = lane; kk < L; kk += 64)
                if (!used[kk]) {
                    kn = kk;
                    break;
                }
            kn = wave_min(kn);
            if (kn >= L) break;
        }
        k = kn;
    }
    if (lane == 0) {
        res.rank = ell;
        res.capped = capped;
        res.zero_faces = zero_faces;
        q.out[blk] = res;
    }
}

// Compressed blocks' faces and fibres -> the operator's arenas; dense blocks -> the compact
// dense arena.  One workgroup per block of the chunk.
template <class FT>
__global__ void __launch_bounds__(256) near_aca_pack_kernel(NearAcaArgs q, const FT *near,
                                                            const FT *faces, const NearBlockDev *dst,
                                                            FT *face_arena, double2 *fib_arena,
                                                            FT *dense_arena) {
    const int blk = blockIdx.x;
    const NearBlockDev S = q.blocks[q.b0 + blk], D = dst[q.b0 + blk];
    const int mn = S.m * S.n, L = q.L;
    if (D.comp) {
        const FT *Hs = faces + (int64_t)blk * q.rc * q.mnmax;
        const double2 *Fs = q.fib + (int64_t)blk * q.rc * L;
        for (int64_t t = threadIdx.x; t < (int64_t)D.crank * mn; t += 256) {
            const int p = (int)(t / mn), e = (int)(t - (int64_t)p * mn);
            face_arena[D.off + t] = Hs[(int64_t)p * q.mnmax + e];
        }
        for (int64_t t = threadIdx.x; t < (int64_t)D.crank * L; t += 256) fib_arena[D.foff + t] = Fs[t];
    } else {
        // dense block: copy the m L n entries
        for (int64_t t = threadIdx.x; t < (int64_t)mn * L; t += 256) dense_arena[D.off + t] = near[S.off + t];
    }
}

// Dense [m][L][n] reconstruction of one compressed block (export): sum_l H_l (x) f_l.
template <class FT>
__global__ void near_aca_expand_kernel(NearBlockDev D, int L, const FT *face_arena,
                                       const double2 *fib_arena, double2 *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int mn = D.m * D.n;
    if (t >= (int64_t)mn * L) return;
    const int i = (int)(t / ((int64_t)L * D.n));
    const int rest = (int)(t - (int64_t)i * L * D.n);
    const int k = rest / D.n, j = rest - k * D.n;
    double2 s = make_double2(0.0, 0.0);
    for (int p = 0; p < D.crank; ++p) {
        const double2 v = cmulq(to_d2(face_arena[D.off + (int64_t)p * mn + i * D.n + j]),
                                fib_arena[D.foff + (int64_t)p * L + k]);
        s.x += v.x;
        s.y += v.y;
    }
    out[t] = s;
}

}  // namespace

void launch_near_aca(const NearAcaArgs &q, int nblk, const void *near, void *faces, int fp32,
                     hipStream_t st) {
    if (nblk <= 0) return;
    if (fp32)
        near_aca_kernel<float2><<<nblk, 64, 0, st>>>(q, (const float2 *)near, (float2 *)faces);
    else
        near_aca_kernel<double2><<<nblk, 64, 0, st>>>(q, (const double2 *)near, (double2 *)faces);
}

void launch_near_aca_pack(const NearAcaArgs &q, int nblk, const void *near, const void *faces,
                          const NearBlockDev *dst, void *face_arena, double2 *fib_arena,
                          void *dense_arena, int fp32, hipStream_t st) {
    if (nblk <= 0) return;
    if (fp32)
        near_aca_pack_kernel<float2><<<nblk, 256, 0, st>>>(q, (const float2 *)near, (const float2 *)faces, dst,
                                                         (float2 *)face_arena, fib_arena, (float2 *)dense_arena);
    else
        near_aca_pack_kernel<double2><<<nblk, 256, 0, st>>>(q, (const double2 *)near, (const double2 *)faces, dst,
                                                          (double2 *)face_arena, fib_arena, (double2 *)dense_arena);
}

void launch_near_aca_expand(const NearBlockDev &D, int L, const void *face_arena,
                            const double2 *fib_arena, double2 *out, int fp32, hipStream_t st) {
    const int64_t n = (int64_t)D.m * D.n * L;
    if (n <= 0) return;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (fp32) near_aca_expand_kernel<float2><<<g, 256, 0, st>>>(D, L, (const float2 *)face_arena, fib_arena, out);
    else near_aca_expand_kernel<double2><<<g, 256, 0, st>>>(D, L, (const double2 *)face_arena, fib_arena, out);
}

}  // namespace gaca
