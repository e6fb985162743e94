// mech_math.h -- FP64 elementary functions of the mechanism kernels.
//
// Device code of the kernels, also compiled for the host by the accuracy test
// (tests/math_host.cpp), which defines MECH_HD_INLINE itself.
#pragma once
#include <math.h>

#ifndef MECH_HD_INLINE
#define MECH_HD_INLINE __host__ __device__ __forceinline__
#endif

namespace mech {

// e^x, e^x - 1 and ln x in FP64 for the rate and reversal-potential
// expressions.  The library versions keep their polynomial coefficients in
// about forty vector registers across the fused kernels' loops, which held
// the FP64 fused kernel at 4 waves per SIMD; these take each coefficient as
// the scalar operand of the fused multiply-add (fma_s), so the kernels fit
// in 79 (FP64) and 71 (FP32-mixed) registers.
// a b + c with c in a scalar register pair (one scalar operand is allowed per
// vector instruction).
MECH_HD_INLINE double fma_s(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
#else
    return fma(a, b, c);   // host builds (the accuracy test): the same operation
#endif
}
// Reduction after Cody and Waite: x = k ln2 + r with k = rint(x / ln2) and r
// formed by two fused multiply-adds against ln2 split into a double and its
// remainder, so |r| <= ln2/2 up to rounding.  e^r - 1 is its Taylor series
// to r^13/13!, whose tail stays below 2^-55 relative to r.  x is first
// clamped to [-746, 710], beyond which e^x is 0 or +inf anyway (NaN passes
// unchanged).  Against long-double references (tests/test_math_accuracy.py):
// e^x within 1 ulp, e^x - 1 within 1.8 ulp, ln x within 1.2 ulp, sin x within
// 1.5 ulp.
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56, kLog2e = 0x1.71547652b82fep+0;
MECH_HD_INLINE double em1_series(double r) {
    double p = 1.0 / 6227020800.0;   // 1/13!, then 1/12! ... 1/3!
    p = fma_s(p, r, 1.0 / 479001600.0);
    p = fma_s(p, r, 1.0 / 39916800.0);
    p = fma_s(p, r, 1.0 / 3628800.0);
    p = fma_s(p, r, 1.0 / 362880.0);
    p = fma_s(p, r, 1.0 / 40320.0);
    p = fma_s(p, r, 1.0 / 5040.0);
    p = fma_s(p, r, 1.0 / 720.0);
    p = fma_s(p, r, 1.0 / 120.0);
    p = fma_s(p, r, 1.0 / 24.0);
    p = fma_s(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    return fma(r * r, p, r);
}
MECH_HD_INLINE int exp_reduce(double x, double &r) {
    x = x < -746.0 ? -746.0 : (x > 710.0 ? 710.0 : x);
    const double k = rint(x * kLog2e);
    r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
    return (int)k;
}
MECH_HD_INLINE double exp_d(double x) {
    double r;
    const int k = exp_reduce(x, r);
    return ldexp(1.0 + em1_series(r), k);
}
// e^x - 1 = 2^k (e^r - 1) + (2^k - 1): the series alone when k = 0, so the
// result keeps its relative accuracy near x = 0.
MECH_HD_INLINE double expm1_d(double x) {
    double r;
    const int k = exp_reduce(x, r);
    return ldexp(em1_series(r), k) + (ldexp(1.0, k) - 1.0);
}
// ln x = e ln2 + ln m with x = m 2^e, m in [sqrt(1/2), sqrt(2)).  With
// f = m - 1 (exact) and s = f/(m + 1), |s| <= 0.172, ln m = 2 atanh(s) =
// 2s + s R with R = 2s^2/3 + 2s^4/5 + ... (series to s^22, tail below 2^-59
// relative), and 2s = f - s f, so ln m = f - s (f - R): the exact f carries
// the result and the rounding of the rest stays small beside it.  0 gives
// -inf, negative arguments and NaN give NaN, +inf gives +inf.
MECH_HD_INLINE double log_d(double x) {
    int e;
    double m = frexp(x, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {   // sqrt(1/2)
        m += m;
        e -= 1;
    }
    const double f = m - 1.0;
    const double s = f / (m + 1.0), z = s * s;
    double p = 2.0 / 23.0;            // then 2/21 ... 2/5
    p = fma_s(p, z, 2.0 / 21.0);
    p = fma_s(p, z, 2.0 / 19.0);
    p = fma_s(p, z, 2.0 / 17.0);
    p = fma_s(p, z, 2.0 / 15.0);
    p = fma_s(p, z, 2.0 / 13.0);
    p = fma_s(p, z, 2.0 / 11.0);
    p = fma_s(p, z, 2.0 / 9.0);
    p = fma_s(p, z, 2.0 / 7.0);
    p = fma_s(p, z, 2.0 / 5.0);
    p = fma_s(p, z, 2.0 / 3.0);
    const double lm = fma(-s, f - z * p, f);
    const double de = (double)e;
    const double y = fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
    if (x > 0.0 && x < INFINITY) return y;
    return x == 0.0 ? -INFINITY : (x == INFINITY ? INFINITY : NAN);
}
// sin x for the clamp waveform: x = k pi/2 + r with k = rint(2x/pi) and r
// formed by three fused multiply-adds against pi/2 split into three doubles
// (accurate while |k| stays far below 2^50), |r| <= pi/4; sin r and cos r
// by their Taylor series to r^19/19! and r^18/18!, and the quadrant k mod 4
// picks +-sin r or +-cos r.  Written out for the same reason as exp_d (the
// library sine holds a large reduction table and its registers).
MECH_HD_INLINE double sin_d(double x) {
    const double k = rint(x * 0x1.45f306dc9c883p-1);   // 2/pi
    double r = fma(-k, 0x1.921fb54442d18p+0, x);
    r = fma(-k, 0x1.1a62633145c07p-54, r);
    r = fma(-k, -0x1.f1976b7ed8fbcp-110, r);
    const double z = r * r;
    double ps = -1.0 / 121645100408832000.0;   // -1/19!, then 1/17! ... 1/5!
    ps = fma_s(ps, z, 1.0 / 355687428096000.0);
    ps = fma_s(ps, z, -1.0 / 1307674368000.0);
    ps = fma_s(ps, z, 1.0 / 6227020800.0);
    ps = fma_s(ps, z, -1.0 / 39916800.0);
    ps = fma_s(ps, z, 1.0 / 362880.0);
    ps = fma_s(ps, z, -1.0 / 5040.0);
    ps = fma_s(ps, z, 1.0 / 120.0);
    ps = fma(ps, z, -1.0 / 6.0);
    const double sr = fma(r * z, ps, r);
    double pc = 1.0 / 6402373705728000.0;   // 1/18!, then -1/16! ... -1/4!
    pc = fma_s(pc, z, -1.0 / 20922789888000.0);
    pc = fma_s(pc, z, 1.0 / 87178291200.0);
    pc = fma_s(pc, z, -1.0 / 479001600.0);
    pc = fma_s(pc, z, 1.0 / 3628800.0);
    pc = fma_s(pc, z, -1.0 / 40320.0);
    pc = fma_s(pc, z, 1.0 / 720.0);
    pc = fma_s(pc, z, -1.0 / 24.0);
    pc = fma(pc, z, 0.5);   // now 1/2 - z/24 + ...
    const double cr = fma(-z, pc, 1.0);
    const double q = k - 4.0 * floor(k * 0.25);   // k mod 4, exact
    const double y = (q == 0.0 || q == 2.0) ? sr : cr;
    return (q >= 2.0) ? -y : y;
}

}  // namespace mech
