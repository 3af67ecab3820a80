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

#include <mutex>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

// ---------------------------------------------------------------------------------------
// Workspace of the allocation-free apply: one fixed array per device, alive until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host code the name
// is a host-side stand-in): it uses the device address that hipGetSymbolAddress returns,
// taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_addr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
    return hipSuccess;
}

void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_addr[device];
}

// Per-block workspace offsets of the VALU apply from the block metadata (what the host
// computes for the allocated workspace): z_off = prefix of sum_rho * nrhs (SUM) or
// sum_rho * L * nrhs (PER_FREQ), t_off = prefix of min(rank, cb) * n * nrhs (SUM; 0 else),
// y_off = prefix of m * nrhs.  One workgroup: each thread sums a contiguous run of blocks,
// the run totals are scanned in LDS, then each thread writes its run's prefixes.
__global__ void __launch_bounds__(1024) apply_offsets_kernel(ApplyDev a, int mode, int cb,
                                                             int64_t *zoff, int64_t *toff,
                                                             int64_t *yoff) {
    __shared__ int64_t sz[1024], st[1024], sy[1024];
    const int nb = a.nfar, t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    const int64_t zmul = mode == 0 ? a.nrhs : (int64_t)a.L * a.nrhs;
    int64_t z = 0, tt = 0, y = 0;
    for (int b = b0; b < b1; ++b) {
        z += (int64_t)a.meta[b].sum_rho * zmul;
        if (mode == 0) tt += (int64_t)min(a.meta[b].rank, cb) * a.far4[4 * b + 3] * a.nrhs;
        y += (int64_t)a.far4[4 * b + 1] * a.nrhs;
    }
    sz[t] = z;
    st[t] = tt;
    sy[t] = y;
    __syncthreads();
    // inclusive scan of the run totals (Hillis-Steele)
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t vz = 0, vt = 0, vy = 0;
        if (t >= d) {
            vz = sz[t - d];
            vt = st[t - d];
            vy = sy[t - d];
        }
        __syncthreads();
        sz[t] += vz;
        st[t] += vt;
        sy[t] += vy;
        __syncthreads();
    }
    z = sz[t] - z;
    tt = st[t] - tt;
    y = sy[t] - y;
    for (int b = b0; b < b1; ++b) {
        zoff[b] = z;
        toff[b] = tt;
        yoff[b] = y;
        z += (int64_t)a.meta[b].sum_rho * zmul;
        if (mode == 0) tt += (int64_t)min(a.meta[b].rank, cb) * a.far4[4 * b + 3] * a.nrhs;
        y += (int64_t)a.far4[4 * b + 1] * a.nrhs;
    }
}

void launch_apply_offsets(const ApplyDev &a, int mode, int cb, int64_t *zoff, int64_t *toff,
                          int64_t *yoff, hipStream_t st) {
    if (a.nfar <= 0) return;
    apply_offsets_kernel<<<1, 1024, 0, st>>>(a, mode, cb, zoff, toff, yoff);
}

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

// SUM: T_l = sum_k f_l[k] X_k[tau] (n x nrhs), z_l = W_l^T T_l for every cross of block b,
// a.apply_cb (<= kApplyCB) crosses at a time: each X_k[tau] element is read once per group
// of crosses (the group size keeps the T workspace within its budget), and
// z_l's rows are dot products over j taken by 8 lanes each (W rows read in order, partial
// sums added by a fixed butterfly).
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
    if (mode == 0) {
        constexpr int CB = kApplyCB;
        __shared__ int64_t s_w[CB], s_z[CB];
        __shared__ int s_rho[CB + 1];
        __shared__ XT s_f[CB * kApplyKF];
        const int nt = n * nr;
        int64_t zo = 0;
        const int cbr = max(1, min(CB, a.apply_cb));
        for (int cg = 0; cg < mt.rank; cg += cbr) {
            const int cb = min(cbr, mt.rank - cg);
            __syncthreads();
            if (threadIdx.x == 0) {
                int rows = 0;
                for (int c = 0; c < cb; ++c) {
                    const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + cg + c];
                    s_w[c] = a.cross_off[(int64_t)b * a.rcap + cg + c] + (int64_t)cm.rho * m;
                    s_z[c] = zo;
                    s_rho[c] = rows;
                    rows += cm.rho;
                    zo += (int64_t)cm.rho * nr;
                }
                s_rho[cb] = rows;
            }
            // T_c for the crosses of the group ([c][j][rhs]); the fibres pass through LDS
            // kApplyKF frequencies at a time.  Blocks with few columns split the frequencies
            // over G adjacent lanes per (j, rhs) (G a power of two, G nt <= workgroup), whose
            // sums are added by a fixed butterfly
            int G = 1;
            while (G < 16 && 2 * G * nt <= (int)blockDim.x) G *= 2;
            const int tpp = (int)blockDim.x / G, gl = (int)threadIdx.x % G;
            for (int t0 = 0; t0 < nt; t0 += tpp) {
                const int t = t0 + (int)threadIdx.x / G;
                const int j = t / nr, cc = t - j * nr;
                const XT *xp = Xp + (int64_t)(c0 + min(j, n - 1)) * nr + cc;
                XT acc[CB];
#pragma unroll
                for (int c = 0; c < CB; ++c) acc[c] = czero<XT>();
                for (int k0 = 0; k0 < L; k0 += kApplyKF) {
                    const int nk = min(kApplyKF, L - k0);
                    __syncthreads();
                    for (int i = threadIdx.x; i < cb * nk; i += blockDim.x) {
                        const int c = i / nk, kk = i - c * nk;
                        s_f[c * kApplyKF + kk] = cast_c<XT>(F[(int64_t)(cg + c) * L + k0 + kk]);
                    }
                    __syncthreads();
#pragma unroll 8
                    for (int kk = gl; kk < nk; kk += G) {
                        const XT x = xp[(int64_t)(k0 + kk) * M * nr];
#pragma unroll
                        for (int c = 0; c < CB; ++c)
                            if (c < cb) acc[c] = cfma(s_f[c * kApplyKF + kk], x, acc[c]);
                    }
                }
                for (int o = G >> 1; o > 0; o >>= 1)
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        acc[c].x += __shfl_xor(acc[c].x, o, 64);
                        acc[c].y += __shfl_xor(acc[c].y, o, 64);
                    }
                if (gl == 0 && t < nt)
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c < cb) T[(int64_t)c * nt + t] = acc[c];
            }
            __syncthreads();
            // z rows (cross c, step q) of the group, 8 lanes per row and right-hand side
            const int rows = s_rho[cb];
            const int l8 = threadIdx.x & 7;
            for (int g = threadIdx.x >> 3; g < rows * nr; g += blockDim.x >> 3) {
                const int ri = g / nr, cc = g - ri * nr;
                int c = 0;
                while (c + 1 < cb && s_rho[c + 1] <= ri) ++c;
                const int q = ri - s_rho[c];
                const FacT *w = arena + s_w[c] + (int64_t)q * n;
                const XT *tc = T + (int64_t)c * nt + cc;
                XT acc = czero<XT>();
#pragma unroll 4
                for (int j = l8; j < n; j += 8) acc = cfma(cast_c<XT>(w[j]), tc[(int64_t)j * nr], acc);
                double ax = acc.x, ay = acc.y;
#pragma unroll
                for (int o = 4; o > 0; o >>= 1) {
                    ax += __shfl_xor(ax, o, 8);
                    ay += __shfl_xor(ay, o, 8);
                }
                if (l8 == 0) {
                    XT r;
                    r.x = ax;
                    r.y = ay;
                    z[s_z[c] + (int64_t)q * nr + cc] = r;
                }
            }
        }
        return;
    }
    int64_t zo = 0;
    for (int c = 0; c < mt.rank; ++c) {
        const CrossMeta cm = a.cmeta[(int64_t)b * a.rcap + c];
        const FacT *W = arena + a.cross_off[(int64_t)b * a.rcap + c] + (int64_t)cm.rho * m;
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
#pragma unroll 8
            for (int qq = 0; qq < cm.rho; ++qq)
                acc = cfma(cast_c<XT>(U[(int64_t)qq * m + r]), z[zo + (int64_t)qq * nr + cc], acc);
            zo += (int64_t)cm.rho * nr;
        }
        ybuf[y_off[b] + t] = acc;
    }
}

// SUM, compressed near blocks: T_l = sum_k f_l[k] X_k[tau] ([crank][n][nrhs]) per block;
// one workgroup per near block (dense ones return at once).
template <class XT>
__global__ void __launch_bounds__(256) apply_near_t_kernel(ApplyDev a, const XT *Xp, XT *tn) {
    const NearBlockDev nb = a.nblocks[blockIdx.x];
    if (!nb.comp || nb.crank == 0) return;
    const int L = a.L, nr = a.nrhs, n = nb.n;
    const int64_t M = a.M;
    const double2 *F = a.near_fib + nb.foff;
    XT *T = tn + a.tn_off[blockIdx.x];
    const int64_t tot = (int64_t)nb.crank * n * nr;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
        const int cc = (int)(t % nr);
        const int64_t rest = t / nr;
        const int j = (int)(rest % n), l = (int)(rest / n);
        const XT *xp = Xp + (int64_t)(nb.c0 + j) * nr + cc;
        XT acc = czero<XT>();
        for (int k = 0; k < L; ++k) acc = cfma(cast_c<XT>(F[(int64_t)l * L + k]), xp[(int64_t)k * M * nr], acc);
        T[t] = acc;
    }
}

// SUM per row: Y[row] = sum over the leaf's near blocks of sum_k N_k[row] X_k + the rows
// y_b of the covering far blocks.  One wave per row: a near block stores row ro as L n
// contiguous entries ([m][L][n]), which the lanes read in order (entry t: frequency t / n,
// column t % n); RC right-hand sides per pass, lane sums added by a fixed-order wave
// reduction.  Grid (leaf, rows / 4).  PART 0: near and far parts; 1: the near part only
// (written to Yp); 2: the far part added to the near part in Yp (1 then 2 gives the values
// of 0 bit for bit, with the far blocks' y computed in between or beside part 1).
template <class NearT, class XT, int RC, int PART>
__global__ void __launch_bounds__(256) apply_leaf_sum_kernel(ApplyDev a, const XT *Xp,
                                                             const XT *ybuf, const int64_t *y_off,
                                                             XT *Yp, const XT *tn) {
    const int leaf = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.y * 4 + wave;
    if (r >= a.leaf_m[leaf]) return;   // the whole wave; no workgroup barrier below
    const int row = a.leaf_r0[leaf] + r;
    const int L = a.L, nr = a.nrhs;
    const int64_t M = a.M;
    const int np0 = a.leaf_near_ptr[leaf], np1 = a.leaf_near_ptr[leaf + 1];
    const int fp0 = a.leaf_far_ptr[leaf], fp1 = a.leaf_far_ptr[leaf + 1];
    const NearT *nearv = a.near64 ? reinterpret_cast<const NearT *>(a.near64)
                                  : reinterpret_cast<const NearT *>(a.near32);
    for (int cr = 0; cr < nr; cr += RC) {
        XT acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] = czero<XT>();
        for (int e = PART == 2 ? np1 : np0; e < np1; ++e) {
            const int ib = a.leaf_near_idx[e];
            const NearBlockDev nb = a.nblocks[ib];
            if (nb.comp) {
                // row ro of sum_l H_l (T_l): entry t = (l, j), H_l row ro at l m n + ro n
                const NearT *fc = reinterpret_cast<const NearT *>(a.near_faces) + nb.off;
                const XT *T = tn + a.tn_off[ib] + cr;
                const int n = nb.n, mn = nb.m * n, ro = row - nb.r0;
                for (int t = lane; t < nb.crank * n; t += 64) {
                    const int l = t / n, j = t - l * n;
                    const XT hv = cast_c<XT>(fc[(int64_t)l * mn + (int64_t)ro * n + j]);
                    const XT *tp = T + (int64_t)t * nr;
#pragma unroll
                    for (int c = 0; c < RC; ++c)
                        if (cr + c < nr) acc[c] = cfma(hv, tp[c], acc[c]);
                }
                continue;
            }
            const int n = nb.n, E = L * n;
            const NearT *base = nearv + nb.off + (int64_t)(row - nb.r0) * E;
            const XT *xb = Xp + (int64_t)nb.c0 * nr + cr;
            // (k, j) of entry t = lane + 64 i, advanced by 64 entries per step; LU entries
            // per round have their loads in flight together and are summed in order
            int k = lane / n, j = lane - k * n;
            const int dk = 64 / n, dj = 64 - dk * n;
            auto step = [&]() {
                k += dk;
                j += dj;
                if (j >= n) {
                    j -= n;
                    ++k;
                }
            };
            constexpr int LU = 8;
            int t = lane;
            for (; t + 64 * (LU - 1) < E; t += 64 * LU) {
                XT nv[LU], xv[LU][RC];
#pragma unroll
                for (int u = 0; u < LU; ++u) {
                    nv[u] = cast_c<XT>(base[t + 64 * u]);
                    const XT *xp = xb + ((int64_t)k * M + j) * nr;
#pragma unroll
                    for (int c = 0; c < RC; ++c) xv[u][c] = cr + c < nr ? xp[c] : czero<XT>();
                    step();
                }
#pragma unroll
                for (int u = 0; u < LU; ++u)
#pragma unroll
                    for (int c = 0; c < RC; ++c)
                        if (cr + c < nr) acc[c] = cfma(nv[u], xv[u][c], acc[c]);
            }
            for (; t < E; t += 64) {
                const XT nv = cast_c<XT>(base[t]);
                const XT *xp = xb + ((int64_t)k * M + j) * nr;
#pragma unroll
                for (int c = 0; c < RC; ++c)
                    if (cr + c < nr) acc[c] = cfma(nv, xp[c], acc[c]);
                step();
            }
        }
        if constexpr (PART != 2) {
#pragma unroll
            for (int c = 0; c < RC; ++c) {
                const double sx = wave_sum((double)acc[c].x), sy = wave_sum((double)acc[c].y);
                acc[c].x = sx;
                acc[c].y = sy;
            }
        }
        if (lane < RC && cr + lane < nr) {
            XT tot = acc[0];
#pragma unroll
            for (int c = 1; c < RC; ++c)
                if (lane == c) tot = acc[c];
            if constexpr (PART == 2) tot = Yp[(int64_t)row * nr + cr + lane];
            if constexpr (PART != 1)
                for (int e = fp0; e < fp1; ++e) {
                    const int b = a.leaf_far_idx[e];
                    tot = cadd(tot, ybuf[y_off[b] + (int64_t)(row - a.far4[4 * b]) * nr + cr + lane]);
                }
            Yp[(int64_t)row * nr + cr + lane] = tot;
        }
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
            if (nb.comp) {
                // sum_l f_l[k] H_l[ro] X_k[tau]
                const NearT *fc = reinterpret_cast<const NearT *>(a.near_faces) + nb.off;
                const XT *xk = Xp + ((int64_t)kf * M + nb.c0) * nr + cc;
                const int mn = nb.m * nb.n;
                for (int l = 0; l < nb.crank; ++l) {
                    XT s = czero<XT>();
                    const NearT *hr = fc + (int64_t)l * mn + (int64_t)ro * nb.n;
                    for (int j = 0; j < nb.n; ++j) s = cfma(cast_c<XT>(hr[j]), xk[(int64_t)j * nr], s);
                    acc = cfma(cast_c<XT>(a.near_fib[nb.foff + (int64_t)l * L + kf]), s, acc);
                }
                continue;
            }
            const NearT *nrow = nearv + nb.off + ((int64_t)ro * L + kf) * nb.n;
            const XT *xk = Xp + ((int64_t)kf * M + nb.c0) * nr + cc;
            for (int j = 0; j < nb.n; ++j) acc = cfma(cast_c<XT>(nrow[j]), xk[(int64_t)j * nr], acc);
        }
        Yp[((int64_t)kf * M + row) * nr + cc] = acc;
    }
}

template <class FacT, class XT, int PART>
static void leaf_sum(const ApplyDev &a, const XT *Xp, const XT *ybuf, const int64_t *y_off, XT *Yp,
                     const XT *tnbuf, hipStream_t st) {
    const dim3 grid(a.nleaf, (a.max_leaf_m + 3) / 4);
    if (a.nrhs == 1)
        apply_leaf_sum_kernel<FacT, XT, 1, PART><<<grid, 256, 0, st>>>(a, Xp, ybuf, y_off, Yp, tnbuf);
    else if (a.nrhs == 2)
        apply_leaf_sum_kernel<FacT, XT, 2, PART><<<grid, 256, 0, st>>>(a, Xp, ybuf, y_off, Yp, tnbuf);
    else
        apply_leaf_sum_kernel<FacT, XT, 4, PART><<<grid, 256, 0, st>>>(a, Xp, ybuf, y_off, Yp, tnbuf);
}

template <class FacT, class XT>
static void apply_impl(const ApplyDev &a, int mode, const XT *X, XT *Y, XT *Xp, XT *Yp, XT *zbuf,
                       XT *tbuf, const int64_t *t_off, XT *ybuf, const int64_t *y_off,
                       hipStream_t st, XT *tnbuf, const ApplySide *side) {
    const int64_t totx = (int64_t)a.L * a.M * a.nrhs;
    permute_x_kernel<XT><<<(unsigned)((totx + 255) / 256), 256, 0, st>>>(X, Xp, a.perm, a.L, a.M,
                                                                          a.nrhs);
    const int nl = mode == 0 ? 1 : a.L;
    if (mode == 0 && side && a.nfar > 0) {
        // far blocks (T, z, y) on the side stream beside the near part of the leaf sums (an
        // L2-bound chain beside an HBM-bound pass), joined before the far parts are added
        GACA_HIP_CHECK(hipEventRecord(side->fork, st));
        GACA_HIP_CHECK(hipStreamWaitEvent(side->stream, side->fork, 0));
        apply_far_a_kernel<FacT, XT><<<a.nfar, 256, 0, side->stream>>>(a, mode, Xp, zbuf, tbuf, t_off);
        apply_far_y_kernel<FacT, XT><<<a.nfar, 256, 0, side->stream>>>(a, zbuf, ybuf, y_off);
        GACA_HIP_CHECK(hipEventRecord(side->join, side->stream));
        if (a.near_faces && a.nnear > 0)
            apply_near_t_kernel<XT><<<a.nnear, 256, 0, st>>>(a, Xp, tnbuf);
        leaf_sum<FacT, XT, 1>(a, Xp, ybuf, y_off, Yp, tnbuf, st);
        GACA_HIP_CHECK(hipStreamWaitEvent(st, side->join, 0));
        leaf_sum<FacT, XT, 2>(a, Xp, ybuf, y_off, Yp, tnbuf, st);
    } else if (mode == 0) {
        if (a.nfar > 0) {
            apply_far_a_kernel<FacT, XT><<<a.nfar, 256, 0, st>>>(a, mode, Xp, zbuf, tbuf, t_off);
            apply_far_y_kernel<FacT, XT><<<a.nfar, 256, 0, st>>>(a, zbuf, ybuf, y_off);
        }
        if (a.near_faces && a.nnear > 0)
            apply_near_t_kernel<XT><<<a.nnear, 256, 0, st>>>(a, Xp, tnbuf);
        leaf_sum<FacT, XT, 0>(a, Xp, ybuf, y_off, Yp, tnbuf, st);
    } else {
        if (a.nfar > 0)
            apply_far_a_kernel<FacT, XT><<<a.nfar, 256, 0, st>>>(a, mode, Xp, zbuf, tbuf, t_off);
        apply_leaf_freq_kernel<FacT, FacT, XT><<<dim3(a.nleaf, nl), 256, 0, st>>>(a, Xp, zbuf, Yp);
    }
    const int64_t toty = (int64_t)nl * a.M * a.nrhs;
    scatter_y_kernel<XT><<<(unsigned)((toty + 255) / 256), 256, 0, st>>>(Yp, Y, a.perm, nl, a.M,
                                                                         a.nrhs);
}

void launch_apply(const ApplyDev &a, int mode, int x_fp32, const void *X, void *Y, void *Xp,
                  void *Yp, void *zbuf, void *tbuf, const int64_t *t_off, void *ybuf,
                  const int64_t *y_off, hipStream_t st, void *tnbuf, const ApplySide *side) {
#define GACA_APPLY(FT, XTT)                                                                  \
    apply_impl<FT, XTT>(a, mode, (const XTT *)X, (XTT *)Y, (XTT *)Xp, (XTT *)Yp, (XTT *)zbuf, \
                        (XTT *)tbuf, t_off, (XTT *)ybuf, y_off, st, (XTT *)tnbuf, side)
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
