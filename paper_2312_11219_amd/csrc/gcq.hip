// History step of the Runge-Kutta gCQ (Sec. 3, temporal discretisation) on the device:
//   eq. (gCQ_xn)      x_{n-1}(s_l) = (I - dt_{n-1} s_l A)^{-1}
//                                    ((b^T A^{-1} x_{n-2}(s_l)) 1 + dt_{n-1} A theta_{n-1}),
//   eq. (gcq_formula) W_l = omega_l (b^T A^{-1} x_{n-1}(s_l)) (I - dt_n s_l A)^{-1} 1,
// per frequency l and spatial unknown j (m-vectors over the stages, complex128).  The
// history term sum_l V(s_l) W_l is then the reordered product of Sec. 4 with the stages as
// right-hand sides.  One thread per (l, j); the m x m complex systems are solved by
// Gaussian elimination with partial pivoting in registers.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace gaca {

namespace {

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// x := (I - z A)^{-1} x for complex z, m <= kGcqMaxStages
__device__ void resolvent_solve(int m, const double *A, double2 z, double2 *x) {
    double2 M[kGcqMaxStages][kGcqMaxStages];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            const double a = A[i * m + j];
            M[i][j] = make_double2((i == j ? 1.0 : 0.0) - z.x * a, -z.y * a);
        }
    for (int c = 0; c < m; ++c) {
        int p = c;
        double best = M[c][c].x * M[c][c].x + M[c][c].y * M[c][c].y;
        for (int r = c + 1; r < m; ++r) {
            const double v = M[r][c].x * M[r][c].x + M[r][c].y * M[r][c].y;
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (p != c) {
            for (int j = 0; j < m; ++j) {
                const double2 t = M[c][j];
                M[c][j] = M[p][j];
                M[p][j] = t;
            }
            const double2 t = x[c];
            x[c] = x[p];
            x[p] = t;
        }
        for (int r = c + 1; r < m; ++r) {
            const double2 f = cdiv2(M[r][c], M[c][c]);
            for (int j = c; j < m; ++j) {
                const double2 t = cmul2(f, M[c][j]);
                M[r][j].x -= t.x;
                M[r][j].y -= t.y;
            }
            const double2 t = cmul2(f, x[c]);
            x[r].x -= t.x;
            x[r].y -= t.y;
        }
    }
    for (int c = m - 1; c >= 0; --c) {
        double2 v = x[c];
        for (int j = c + 1; j < m; ++j) {
            const double2 t = cmul2(M[c][j], x[j]);
            v.x -= t.x;
            v.y -= t.y;
        }
        x[c] = cdiv2(v, M[c][c]);
    }
}

__global__ void __launch_bounds__(256) gcq_history_kernel(GcqDev q, const double *s_re,
                                                          const double *s_im, const double2 *theta,
                                                          double2 *x, double2 *W) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)q.L * q.M) return;
    const int l = (int)(t / q.M);
    const int m = q.m;
    const double2 s = make_double2(s_re[l], s_im[l]);
    double2 v[kGcqMaxStages];
    // g . x_{n-2}, g = b^T A^{-1}
    double2 gx = make_double2(0.0, 0.0);
    for (int i = 0; i < m; ++i) {
        const double2 xi = x[t * m + i];
        gx.x += q.g[i] * xi.x;
        gx.y += q.g[i] * xi.y;
    }
    // right-hand side (g . x_{n-2}) 1 + dt_{n-1} A theta_{n-1}
    const int64_t j = t - (int64_t)l * q.M;
    for (int i = 0; i < m; ++i) {
        double2 a = gx;
        for (int k = 0; k < m; ++k) {
            const double2 th = theta[j * m + k];
            a.x += q.dt_prev * q.A[i * m + k] * th.x;
            a.y += q.dt_prev * q.A[i * m + k] * th.y;
        }
        v[i] = a;
    }
    resolvent_solve(m, q.A, make_double2(q.dt_prev * s.x, q.dt_prev * s.y), v);
    gx = make_double2(0.0, 0.0);
    for (int i = 0; i < m; ++i) {
        x[t * m + i] = v[i];
        gx.x += q.g[i] * v[i].x;
        gx.y += q.g[i] * v[i].y;
    }
    // W_l = omega_l (g . x_{n-1}) (I - dt_n s_l A)^{-1} 1
    for (int i = 0; i < m; ++i) v[i] = make_double2(1.0, 0.0);
    resolvent_solve(m, q.A, make_double2(q.dt_cur * s.x, q.dt_cur * s.y), v);
    const double2 c = cmul2(make_double2(q.w_re[l], q.w_im[l]), gx);
    for (int i = 0; i < m; ++i) W[t * m + i] = cmul2(c, v[i]);
}

}  // namespace

void launch_gcq_history(const GcqDev &q, const double *s_re, const double *s_im,
                        const double2 *theta, double2 *x, double2 *W, hipStream_t st) {
    const int64_t n = (int64_t)q.L * q.M;
    if (n <= 0) return;
    gcq_history_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(q, s_re, s_im, theta, x, W);
}

}  // namespace gaca
