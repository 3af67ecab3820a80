// Device helpers shared by the HIP kernels: double2 complex arithmetic and fixed-order
// wave64 / workgroup reductions (deterministic: the same inputs give the same bits).
#pragma once

#include <hip/hip_runtime.h>

namespace gaca {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {  // c + a * b
    return make_double2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 conj_d2(double2 a) { return make_double2(a.x, -a.y); }

// float2 overloads (mixed-precision faces); cabs2 of a float2 is evaluated in FP64
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
    return make_float2(c.x + a.x * b.x - a.y * b.y, c.y + a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cdiv(float2 a, float2 b) {
    float d = b.x * b.x + b.y * b.y;
    return make_float2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double cabs2(float2 a) {
    return (double)a.x * a.x + (double)a.y * a.y;
}
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
template <class T>
__device__ __forceinline__ T from_d2(double2 a);
template <>
__device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <>
__device__ __forceinline__ float2 from_d2<float2>(double2 a) {
    return make_float2((float)a.x, (float)a.y);
}
template <class T>
__device__ __forceinline__ T cast_c(double2 a) { return from_d2<T>(a); }
template <class T>
__device__ __forceinline__ T cast_c(float2 a);
template <>
__device__ __forceinline__ float2 cast_c<float2>(float2 a) { return a; }
template <>
__device__ __forceinline__ double2 cast_c<double2>(float2 a) { return to_d2(a); }
template <class T>
__device__ __forceinline__ T czero();
template <>
__device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ float2 czero<float2>() { return make_float2(0.0f, 0.0f); }

// Wave64 reductions without LDS: four DPP steps (quad_perm [1,0,3,2] and [2,3,0,1],
// row_half_mirror, row_mirror) leave every lane with the sum (max, min) of its row of 16
// lanes; the four row values are then combined from v_readlane results, so every lane
// gets the same value in a fixed order.  Callers are wave-converged.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp_i<0xB1>(v));
    v = min(v, dpp_i<0x4E>(v));
    v = min(v, dpp_i<0x141>(v));
    v = min(v, dpp_i<0x140>(v));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Workgroup reductions; buf must hold >= 8 * NT / 64 doubles of shared memory.  Each call
// writes the per-wave values into one of two slots (alternating from call to call), passes
// one barrier and reads the slot back: a slot is written again only two calls later, after
// the barrier of the call in between, which every thread reaches only once it has read the
// slot.  Every call holds exactly one barrier.
template <int NT>
struct Red {
    static constexpr int NW = NT / 64;
    double *buf;
    int sl = 0;
    __device__ double *slot() {
        double *b = buf + sl;
        sl ^= 4 * NW;
        return b;
    }
    __device__ double sum(double v) {
        v = wave_sum(v);
        double *b = slot();
        if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += b[w];
        return t;
    }
    __device__ void sum3(double &a, double &bb, double &c) {
        a = wave_sum(a);
        bb = wave_sum(bb);
        c = wave_sum(c);
        double *b = slot();
        if ((threadIdx.x & 63) == 0) {
            b[3 * (threadIdx.x >> 6)] = a;
            b[3 * (threadIdx.x >> 6) + 1] = bb;
            b[3 * (threadIdx.x >> 6) + 2] = c;
        }
        __syncthreads();
        a = bb = c = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            a += b[3 * w];
            bb += b[3 * w + 1];
            c += b[3 * w + 2];
        }
    }
    __device__ double max(double v) {
        v = wave_max(v);
        double *b = slot();
        if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = b[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) t = fmax(t, b[w]);
        return t;
    }
    // sums of a, b, c and max of d in one round (4 NW doubles)
    __device__ void sum3max(double &a, double &bb, double &c, double &d) {
        a = wave_sum(a);
        bb = wave_sum(bb);
        c = wave_sum(c);
        d = wave_max(d);
        double *b = slot();
        if ((threadIdx.x & 63) == 0) {
            double *o = b + 4 * (threadIdx.x >> 6);
            o[0] = a;
            o[1] = bb;
            o[2] = c;
            o[3] = d;
        }
        __syncthreads();
        a = bb = c = 0.0;
        d = b[3];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            a += b[4 * w];
            bb += b[4 * w + 1];
            c += b[4 * w + 2];
            d = fmax(d, b[4 * w + 3]);
        }
    }
    // max of a and sum of b in one round
    __device__ void maxsum(double &a, double &bb) {
        a = wave_max(a);
        bb = wave_sum(bb);
        double *b = slot();
        if ((threadIdx.x & 63) == 0) {
            b[2 * (threadIdx.x >> 6)] = a;
            b[2 * (threadIdx.x >> 6) + 1] = bb;
        }
        __syncthreads();
        a = b[0];
        bb = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            a = fmax(a, b[2 * w]);
            bb += b[2 * w + 1];
        }
    }
    __device__ int imin(int v) {
        v = wave_min(v);
        int *b = reinterpret_cast<int *>(slot());
        if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = v;
        __syncthreads();
        int t = b[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) t = min(t, b[w]);
        return t;
    }
};

// One-wave workgroups: the butterfly shuffles leave every lane with the result, so the
// reductions need neither LDS nor a barrier (same values as the general version).
template <>
struct Red<64> {
    double *buf;
    __device__ double sum(double v) { return wave_sum(v); }
    __device__ void sum3(double &a, double &b, double &c) {
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
    }
    __device__ double max(double v) { return wave_max(v); }
    __device__ void sum3max(double &a, double &b, double &c, double &d) {
        a = wave_sum(a);
        b = wave_sum(b);
        c = wave_sum(c);
        d = wave_max(d);
    }
    __device__ void maxsum(double &a, double &b) {
        a = wave_max(a);
        b = wave_sum(b);
    }
    __device__ int imin(int v) { return wave_min(v); }
};

// sum_{qq in [q0, q1)} a[qq * sa] * b[qq * sb] with NACC independent partial sums, so that
// 2 NACC loads are in flight per thread (the loops are latency-bound otherwise).
template <class T, int NACC = 8>
__device__ __forceinline__ T dot_strided(const T *__restrict__ a, int64_t sa,
                                         const T *__restrict__ b, int64_t sb, int q0, int q1) {
    T s[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) s[t] = czero<T>();
    int qq = q0;
    for (; qq + NACC <= q1; qq += NACC) {
        T av[NACC], bv[NACC];
#pragma unroll
        for (int t = 0; t < NACC; ++t) {
            av[t] = a[(int64_t)(qq + t) * sa];
            bv[t] = b[(int64_t)(qq + t) * sb];
        }
#pragma unroll
        for (int t = 0; t < NACC; ++t) s[t] = cfma(av[t], bv[t], s[t]);
    }
    for (; qq < q1; ++qq) s[0] = cfma(a[(int64_t)qq * sa], b[(int64_t)qq * sb], s[0]);
#pragma unroll
    for (int w = NACC / 2; w > 0; w /= 2)
#pragma unroll
        for (int t = 0; t < w; ++t) s[t] = cadd(s[t], s[t + w]);
    return s[0];
}

}  // namespace gaca
