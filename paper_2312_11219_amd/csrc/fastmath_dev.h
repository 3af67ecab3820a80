// FP64 e^x and sin x, cos x for the kernel evaluations e^{-s r} = e^{-Re(s) r}
// (cos(Im(s) r) - i sin(Im(s) r)) of the Laplace-domain kernels (Sec. 3).
//
// Method: range reduction after Cody and Waite ("Software Manual for the Elementary
// Functions", 1980): x = n c + y with c = ln 2 (e^x) or pi / 2 (sin, cos), n = rint(x / c),
// and c split into a sum of doubles (c1 + c2 [+ c3], each the nearest double to what the
// previous ones leave of c) so that y = x - n c1 - n c2 - n c3 is formed by fused
// multiply-adds with an error of a few units in the last place of y.  Then the Taylor
// polynomials, in Horner form with the coefficients 1 / k! rounded to double:
//   e^y,  |y| <= ln2 / 2, degree 13: remainder below 6e-18 relative;
//   sin y, |y| <= pi / 4, degree 17: remainder below 1e-19;
//   cos y, |y| <= pi / 4, degree 16: remainder below 3e-18.
// e^x = 2^n e^y (ldexp); sin and cos from the quadrant n mod 4.  Outside the ranges where
// the reduction holds (|x| > 2^20 for sin and cos) the library routines are called; e^x is 0
// below -745.2 and +inf above 709.8, as the correctly rounded function.
//
// The constants are the nearest doubles to the exact values (pinned by the host tests,
// which recompute them from ln 2 and pi in 80-digit decimal arithmetic).
#pragma once

#include <cmath>

#ifndef __HIP__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace gaca {
namespace fm {

constexpr double kLog2e = 0x1.71547652b82fep+0;       // 1 / ln 2
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;       // ln 2 = hi + lo
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;   // 2 / pi
constexpr double kPio2A = 0x1.921fb54442d18p+0;       // pi / 2 = a + b + c
constexpr double kPio2B = 0x1.1a62633145c07p-54;
constexpr double kPio2C = -0x1.f1976b7ed8fbcp-110;

// 1 / k!, k = 0 .. 17.  In device code the table lives in the constant address space
// (read with scalar loads into scalar registers): as literals, each addend of a Horner step
// cost two extra vector moves.
#if defined(__HIP_DEVICE_COMPILE__)
static __constant__ double kInvFact[18] = {
#else
constexpr double kInvFact[18] = {
#endif
    0x1.0000000000000p+0,  0x1.0000000000000p+0,  0x1.0000000000000p-1,  0x1.5555555555555p-3,
    0x1.5555555555555p-5,  0x1.1111111111111p-7,  0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13,
    0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
    0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33, 0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-41,
    0x1.ae7f3e733b81fp-45, 0x1.952c77030ad4ap-49};

__host__ __device__ inline double exp(double x) {
    if (x < -745.2) return 0.0;
    if (x > 709.8) return HUGE_VAL;
    const double n = rint(x * kLog2e);
    double y = fma(-n, kLn2Hi, x);
    y = fma(-n, kLn2Lo, y);
    double p = kInvFact[13];
#pragma unroll
    for (int k = 12; k >= 0; --k) p = fma(p, y, kInvFact[k]);
    return ldexp(p, (int)n);
}

// The library's routine for the arguments beyond the reduction's range (and NaN); kept out
// of line so that the common path stays small enough to be inlined into the callers.
struct SinCos {
    double s, c;
};

__host__ __device__ __attribute__((noinline)) inline SinCos sincos_wide(double x) {
    SinCos r;
    ::sincos(x, &r.s, &r.c);
    return r;
}

__host__ __device__ inline void sincos(double x, double *s, double *c) {
    if (!(fabs(x) <= 1048576.0)) {
        const SinCos r = sincos_wide(x);
        *s = r.s;
        *c = r.c;
        return;
    }
    const double n = rint(x * kTwoOverPi);
    double y = fma(-n, kPio2A, x);
    y = fma(-n, kPio2B, y);
    y = fma(-n, kPio2C, y);
    const double y2 = y * y;
    // sin y = y + y^3 (-1/3! + y^2 (1/5! - ...)), cos y = 1 - y^2/2! + ...
    double ts = kInvFact[17];
#pragma unroll
    for (int k = 15; k >= 3; k -= 2) ts = fma(ts, y2, ((k >> 1) & 1) ? -kInvFact[k] : kInvFact[k]);
    const double sy = fma(y * y2, ts, y);
    double tc = kInvFact[16];
#pragma unroll
    for (int k = 14; k >= 0; k -= 2) tc = fma(tc, y2, ((k >> 1) & 1) ? -kInvFact[k] : kInvFact[k]);
    const double cy = tc;
    const int q = (int)n & 3;
    const double sv = (q & 1) ? cy : sy;
    const double cv = (q & 1) ? sy : cy;
    *s = (q & 2) ? -sv : sv;
    *c = ((q + 1) & 2) ? -cv : cv;
}

}  // namespace fm
}  // namespace gaca
