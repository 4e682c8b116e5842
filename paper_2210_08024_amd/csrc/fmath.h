// Double-precision exp and log for the plain (FP64) path.
//
// The device library's exp and log handle every corner of the IEEE range and cost about 50 and
// 110 instructions; the source step calls them some 90 and 20 times per substep and is bound by
// instruction issue.  These versions follow the constructions below, take about 22 and 30
// instructions, and stay within a few ulp over the arguments the step produces.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ism {

// ln 2 split for Cody-Waite reduction: the head keeps 32 significant bits, so k * head is exact
// for |k| < 2^21; head + tail = ln 2 to ~2^-86.
constexpr double LN2_HEAD = 0x1.62e42fee00000p-1;
constexpr double LN2_TAIL = 0x1.a39ef35793c76p-33;

// e^x: x = k ln2 + r with k = rint(x / ln2), |r| <= ln2 / 2; e^r = 1 + r + r^2 g(r) with g a
// degree-9 Chebyshev fit of (e^r - 1 - r) / r^2 on |r| <= 0.35 (coefficients from
// fmath_fit.py; 0.18 ulp over the interval), in Horner form; the result scaled by 2^k.
// Arguments outside [-746, 710] saturate (to 0 and inf) through a max and a min, which also
// send a NaN argument to the lower bound: a NaN state shows in the step's other terms.
__host__ __device__ __forceinline__ double fexp(double x) {
  x = __builtin_fmin(__builtin_fmax(x, -746.0), 710.0);
  // k = rint(x / ln2) by the 1.5 2^52 shift: the sum keeps k in its low mantissa bits, so the
  // integer for the scaling is the low word of kd as it stands (|k| < 2^31 after the clamp)
  const double kd = fma(x, 1.4426950408889634074, 0x1.8p52);
  const double k = kd - 0x1.8p52;
  double r = fma(-k, LN2_HEAD, x);
  r = fma(-k, LN2_TAIL, r);
  double p = 0x1.af3cd7b3560d9p-26;
  p = fma(p, r, 0x1.2894eb03786e2p-22);
  p = fma(p, r, 0x1.71de0be80e7e8p-19);
  p = fma(p, r, 0x1.a019b62aaa671p-16);
  p = fma(p, r, 0x1.a01a01a83a3a3p-13);
  p = fma(p, r, 0x1.6c16c1794bd5cp-10);
  p = fma(p, r, 0x1.111111111091ap-7);
  p = fma(p, r, 0x1.5555555553b72p-5);
  p = fma(p, r, 0x1.5555555555556p-3);
  p = fma(p, r, 0x1.0000000000001p-1);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)(uint32_t)__builtin_bit_cast(uint64_t, kd));
}

// e^x - 1: for |x| <= 0.35 the same fit as fexp without its leading 1 (x + x^2 g(x)), so small
// arguments keep full relative precision; elsewhere fexp(x) - 1, where the subtraction loses at
// most a bit (|e^x - 1| > 0.29 there).
__host__ __device__ __forceinline__ double fexpm1(double x) {
  if (!(fabs(x) <= 0.35)) return fexp(x) - 1.0;
  double p = 0x1.af3cd7b3560d9p-26;
  p = fma(p, x, 0x1.2894eb03786e2p-22);
  p = fma(p, x, 0x1.71de0be80e7e8p-19);
  p = fma(p, x, 0x1.a019b62aaa671p-16);
  p = fma(p, x, 0x1.a01a01a83a3a3p-13);
  p = fma(p, x, 0x1.6c16c1794bd5cp-10);
  p = fma(p, x, 0x1.111111111091ap-7);
  p = fma(p, x, 0x1.5555555553b72p-5);
  p = fma(p, x, 0x1.5555555555556p-3);
  p = fma(p, x, 0x1.0000000000001p-1);
  return fma(x * x, p, x);
}

// Seed of the reciprocal: the hardware's on the device; on the host (where the checks of this
// file run) 1 / b rounded to float precision, no better than the hardware's, so that the
// refinement below is what those checks exercise.
__host__ __device__ __forceinline__ double rcp_seed(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(b);
#else
  int e;
  const double m = frexp(b, &e);
  return ldexp((double)(1.0f / (float)m), -e);
#endif
}

// a / b for b a finite positive number in [2^-1000, 2^1000] (each caller bounds its denominator
// there): the seed refined by two Newton steps r' = r + r (1 - b r), each doubling its correct
// bits, times a -- the reciprocal-based form, without the range scaling and final correction of
// the general division (6 instructions against 11); within two ulp of a / b.
__host__ __device__ __forceinline__ double fdivp(double a, double b) {
  double r = rcp_seed(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
}

// The same with one correction of the quotient, q' = q + r (a - b q): within an ulp (8
// instructions); the log's reduced argument takes this one.
__host__ __device__ __forceinline__ double fdivp1(double a, double b) {
  double r = rcp_seed(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// ln x: x = 2^e m with m in [sqrt(1/2), sqrt(2)); with f = m - 1 (exact) and s = f / (2 + f),
// ln m = 2 atanh s = 2 s + s z p(z), z = s^2 <= 0.02944, with p a degree-6 Chebyshev fit of
// 2 (atanh s - s) / s^3 on z <= 0.0295 (coefficients from fmath_fit.py; 0.04 ulp);
// ln x = e ln2 + ln m.  flogp takes a positive finite normal x (its callers' arguments are);
// flog adds the special cases: 0 gives -inf, +inf gives +inf, negative arguments and NaN give NaN.
__host__ __device__ __forceinline__ double flogp(double x) {
  int e;
  double m = frexp(x, &e);  // m in [0.5, 1)
  const bool lo = m < 0.70710678118654752440;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double f = m - 1.0;
  const double s = fdivp1(f, 2.0 + f);
  const double z = s * s;
  double p = 0x1.2b6776a1bf0b9p-3;
  p = fma(p, z, 0x1.39fd25d62ab23p-3);
  p = fma(p, z, 0x1.7462be245eae3p-3);
  p = fma(p, z, 0x1.c71c62c42db89p-3);
  p = fma(p, z, 0x1.2492492e0b70cp-2);
  p = fma(p, z, 0x1.99999999951f5p-2);
  p = fma(p, z, 0x1.5555555555558p-1);
  const double lm = fma(s * z, p, s + s);
  const double de = (double)e;
  return fma(de, LN2_HEAD, fma(de, LN2_TAIL, lm));
}

__host__ __device__ __forceinline__ double flog(double x) {
  const double r = flogp(x);
  const double inf = __builtin_huge_val();
  return (x > 0.0 && x < inf) ? r : (x == 0.0 ? -inf : (x == inf ? inf : __builtin_nan("")));
}

}  // namespace ism
