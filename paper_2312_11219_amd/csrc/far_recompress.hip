// Recompression of the face factors after the face ACA (Sec. 4, remarks for the
// implementation): U W^T = Q_U (R_U R_W^T) Q_W^T with U = Q_U R_U, W = Q_W R_W; the SVD of
// the small core K = R_U R_W^T = X Sigma Y^H gives the SVD-like form, truncated while the
// dropped singular values stay within the face tolerance,
//   sqrt(sum of dropped sigma^2) <= eps_aca sqrt(ref2 + sum sigma^2),  at least one kept,
// where ref2 = ||C^(l-1)(:,:,k)||_F^2 (the face ACA's own reference).  The stored factors
// become U' = Q_U X_r Sigma_r and W' = Q_W conj(Y_r), computed without any inverse of R:
//   U' = U R_W^T Y_r,   W' = W R_U^T conj(X_r Sigma_r) Sigma_r^{-2}
// (K Y_r = X_r Sigma_r and X_r^H K = Sigma_r Y_r^H).
//
// R_U, R_W: Cholesky factors of the column-scaled Gram matrices D^{-1} U^H U D^{-1}
// (D = column norms; a non-positive pivot marks a dependent column, whose row of R is
// zero); the SVD of K by one-sided (Hestenes) Jacobi rotations on its columns, round-robin
// pairs, until a sweep rotates no pair with |k_p^H k_q| > 1e-15 ||k_p|| ||k_q||.  All in
// FP64 (the mixed path's FP32 factors are widened and the results rounded back).
// Faces of rank 1 are already in that form; faces of rank above kRecMaxRank are kept as
// computed.  One workgroup per face, grid-stride over the active faces, each workgroup with
// its own slot of 6 kRecMaxRank^2 complex doubles of workspace (R_U, R_W, K, V, A_U, B_W);
// the old factors are copied to the face's H slot (m n >= rho max(m, n)) while the new
// ones are written in place.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

namespace {

template <bool MIXED>
using rface_t = typename std::conditional<MIXED, float2, double2>::type;

__device__ __forceinline__ double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {   // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Gram matrix G[p][q] = sum_i conj(F[p][i]) F[q][i] (rows p, q of the stored factor, length
// len), full Hermitian, column-major ld = rho; one wave per entry of the upper triangle.
template <class FT>
__device__ void gram(const FT *F, int rho, int len, double2 *G) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int npair = rho * (rho + 1) / 2;
    for (int t = wave; t < npair; t += 4) {
        int p = 0, rem = t;
        while (rem >= rho - p) {
            rem -= rho - p;
            ++p;
        }
        const int q = p + rem;
        double sr = 0.0, si = 0.0;
        for (int i = lane; i < len; i += 64) {
            const double2 v = cconjmul(to_d2(F[(int64_t)p * len + i]), to_d2(F[(int64_t)q * len + i]));
            sr += v.x;
            si += v.y;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) {
            G[q * rho + p] = make_double2(sr, si);    // (p, q), column-major
            G[p * rho + q] = make_double2(sr, -si);   // (q, p)
        }
    }
    __syncthreads();
}

// In place: G (Hermitian PSD, column-major) -> upper Cholesky factor R with R^H R = G,
// computed on the column-scaled matrix and scaled back (R = R^ D).
__device__ void cholesky_upper(double2 *G, int rho, double *dsc) {
    const int tid = threadIdx.x;
    for (int q = tid; q < rho; q += 256) dsc[q] = sqrt(fmax(G[q * rho + q].x, 0.0));
    __syncthreads();
    for (int e = tid; e < rho * rho; e += 256) {
        const int p = e % rho, q = e / rho;
        const double s = dsc[p] * dsc[q];
        G[e] = s > 0.0 ? make_double2(G[e].x / s, G[e].y / s) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    __shared__ double piv;
    for (int j = 0; j < rho; ++j) {
        if (tid == 0) {
            double a = G[j * rho + j].x;
            for (int k = 0; k < j; ++k) a -= cabs2(G[j * rho + k]);   // R[k][j] stored at (k, j)
            piv = a > 1e-14 ? sqrt(a) : 0.0;
        }
        __syncthreads();
        const double r = piv;
        // row j of R: R[j][c] = (G[j][c] - sum_k conj(R[k][j]) R[k][c]) / R[j][j], c > j
        for (int c = j + 1 + tid; c < rho; c += 256) {
            double2 v = G[c * rho + j];
            for (int k = 0; k < j; ++k) {
                const double2 t = cconjmul(G[j * rho + k], G[c * rho + k]);
                v.x -= t.x;
                v.y -= t.y;
            }
            G[c * rho + j] = r > 0.0 ? make_double2(v.x / r, v.y / r) : make_double2(0.0, 0.0);
        }
        if (tid == 0) G[j * rho + j] = make_double2(r, 0.0);
        __syncthreads();
    }
    // strictly lower part to zero, columns scaled back by D
    for (int e = tid; e < rho * rho; e += 256) {
        const int p = e % rho, q = e / rho;
        G[e] = p > q ? make_double2(0.0, 0.0) : make_double2(G[e].x * dsc[q], G[e].y * dsc[q]);
    }
    __syncthreads();
}

}  // namespace

template <bool MIXED>
__global__ void __launch_bounds__(256) far_recompress_kernel(AcaParams P, FarBatchDev bd,
                                                             const FarActive *act, int nact,
                                                             double2 *ws) {
    using FT = rface_t<MIXED>;
    constexpr int RM = kRecMaxRank;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double2 *RU = ws + (int64_t)blockIdx.x * kRecSlot;
    double2 *RW = RU + RM * RM, *K = RW + RM * RM, *V = K + RM * RM, *AU = V + RM * RM,
            *BW = AU + RM * RM;
    __shared__ double dsc[RM], sig2[RM];
    __shared__ int order[RM], rkeep, any_rot;
    for (int a = blockIdx.x; a < nact; a += gridDim.x) {
        const FarActive A = act[a];
        const int b = A.b;
        const int rho = bd.st[b].rho;
        if (rho < 2 || rho > RM) continue;
        const FarBlockDev B = bd.blk[b];
        const int m = B.m, n = B.n;
        FT *U = reinterpret_cast<FT *>(bd.uw) + B.uw_off;
        FT *W = U + (int64_t)B.rho_max * m;
        FT *tmp = reinterpret_cast<FT *>(bd.hpool) + A.hslot;   // m n >= rho max(m, n)
        gram(U, rho, m, RU);
        gram(W, rho, n, RW);
        cholesky_upper(RU, rho, dsc);
        cholesky_upper(RW, rho, dsc);
        // K = R_U R_W^T, V = I (column-major)
        for (int e = tid; e < rho * rho; e += 256) {
            const int p = e % rho, q = e / rho;
            double2 s = make_double2(0.0, 0.0);
            for (int k = max(p, q); k < rho; ++k) {   // R upper: R_U[p][k] needs k >= p, R_W[q][k] needs k >= q
                const double2 t = cmul_d(RU[k * rho + p], RW[k * rho + q]);
                s.x += t.x;
                s.y += t.y;
            }
            K[e] = s;
            V[e] = make_double2(p == q ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        // one-sided Jacobi: round-robin pairs over rp = rho rounded up to even
        const int rp = rho + (rho & 1);
        for (int sweep = 0; sweep < 40; ++sweep) {
            if (tid == 0) any_rot = 0;
            __syncthreads();
            for (int round = 0; round < rp - 1; ++round) {
                for (int pr = wave; pr < rp / 2; pr += 4) {
                    // positions pr and rp - 1 - pr of the circle; position 0 fixed
                    auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (rp - 1); };
                    int p = at(pr), q = at(rp - 1 - pr);
                    if (p > q) {
                        const int t = p;
                        p = q;
                        q = t;
                    }
                    if (q >= rho) continue;   // padding column
                    double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
                    for (int i = lane; i < rho; i += 64) {
                        const double2 kp = K[p * rho + i], kq = K[q * rho + i];
                        al += cabs2(kp);
                        be += cabs2(kq);
                        const double2 t = cconjmul(kp, kq);
                        gr += t.x;
                        gi += t.y;
                    }
                    al = wave_sum(al);
                    be = wave_sum(be);
                    gr = wave_sum(gr);
                    gi = wave_sum(gi);
                    const double gab = sqrt(gr * gr + gi * gi);
                    if (!(gab > 1e-15 * sqrt(al * be))) continue;
                    if (lane == 0) any_rot = 1;
                    // k_q <- e^{-i phi} k_q makes the product real; then a real rotation
                    const double2 ph = make_double2(gr / gab, -gi / gab);   // e^{-i phi}
                    const double zeta = (be - al) / (2.0 * gab);
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                    for (int i = lane; i < rho; i += 64) {
                        const double2 kp = K[p * rho + i], kq = cmul_d(K[q * rho + i], ph);
                        K[p * rho + i] = make_double2(c * kp.x - s * kq.x, c * kp.y - s * kq.y);
                        K[q * rho + i] = make_double2(s * kp.x + c * kq.x, s * kp.y + c * kq.y);
                        const double2 vp = V[p * rho + i], vq = cmul_d(V[q * rho + i], ph);
                        V[p * rho + i] = make_double2(c * vp.x - s * vq.x, c * vp.y - s * vq.y);
                        V[q * rho + i] = make_double2(s * vp.x + c * vq.x, s * vp.y + c * vq.y);
                    }
                }
                __syncthreads();
            }
            if (!any_rot) break;
            __syncthreads();
        }
        // singular values (column norms of K V), order by decreasing value (ties: index)
        for (int q = wave; q < rho; q += 4) {
            double s2 = 0.0;
            for (int i = lane; i < rho; i += 64) s2 += cabs2(K[q * rho + i]);
            s2 = wave_sum(s2);
            if (lane == 0) sig2[q] = s2;
        }
        __syncthreads();
        for (int q = tid; q < rho; q += 256) {
            int r = 0;
            for (int x = 0; x < rho; ++x) r += sig2[x] > sig2[q] || (sig2[x] == sig2[q] && x < q);
            order[r] = q;
        }
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            for (int r = 0; r < rho; ++r) tot += sig2[order[r]];
            const double lim2 = P.eps_aca * P.eps_aca * (bd.st[b].ref2 + tot);
            int r = rho;
            double tail = 0.0;
            while (r > 1 && tail + sig2[order[r - 1]] <= lim2) {
                tail += sig2[order[r - 1]];
                --r;
            }
            rkeep = r;
        }
        __syncthreads();
        const int rk = rkeep;
        // A_U = R_W^T V_r and B_W = R_U^T conj((K V)_r) Sigma_r^{-2} (rho x rk, column-major)
        for (int e = tid; e < rho * rk; e += 256) {
            const int k = e % rho, c = e / rho, oc = order[c];
            double2 au = make_double2(0.0, 0.0), bw = make_double2(0.0, 0.0);
            for (int q = 0; q <= k; ++q) {
                const double2 t = cmul_d(RW[k * rho + q], V[oc * rho + q]);
                au.x += t.x;
                au.y += t.y;
                const double2 u = cmul_d(RU[k * rho + q], conj_d2(K[oc * rho + q]));
                bw.x += u.x;
                bw.y += u.y;
            }
            const double is2 = 1.0 / sig2[oc];
            AU[c * rho + k] = au;
            BW[c * rho + k] = make_double2(bw.x * is2, bw.y * is2);
        }
        // U' = U A_U and W' = W B_W, through a copy of the old factor in the face's H slot
        auto apply = [&](FT *F, int len, const double2 *Tm) {
            for (int64_t e = tid; e < (int64_t)rho * len; e += 256) tmp[e] = F[e];
            __syncthreads();
            for (int64_t e = tid; e < (int64_t)rk * len; e += 256) {
                const int c = (int)(e / len), i = (int)(e - (int64_t)c * len);
                double2 acc = make_double2(0.0, 0.0);
                for (int k = 0; k < rho; ++k) {
                    const double2 t = cmul_d(to_d2(tmp[(int64_t)k * len + i]), Tm[c * rho + k]);
                    acc.x += t.x;
                    acc.y += t.y;
                }
                F[e] = from_d2<FT>(acc);
            }
            __syncthreads();
        };
        apply(U, m, AU);
        apply(W, n, BW);
        if (tid == 0) bd.st[b].rho = rk;
        __syncthreads();
    }
}

void launch_far_recompress(const AcaParams &P, const FarBatchDev &bd, const FarActive *act,
                           int nact, double2 *ws, int nslot, hipStream_t st) {
    if (nact <= 0) return;
    const int g = nact < nslot ? nact : nslot;
    if (bd.mixed) far_recompress_kernel<true><<<g, 256, 0, st>>>(P, bd, act, nact, ws);
    else far_recompress_kernel<false><<<g, 256, 0, st>>>(P, bd, act, nact, ws);
}

}  // namespace gaca
