// vsh_math.hpp -- natural logarithm for the shower's hot loop.
//
// x = 2^e m with m in [1/sqrt2, sqrt2); ln x = e ln2 + ln m and
// ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 3 - 2 sqrt2 < 0.1716,
// summed as the odd Taylor series 2 (s + s^3/3 + ... + s^21/21): the first
// omitted term is below 2^-58 of the sum.  m - 1 is exact (Sterbenz), so the
// result keeps its relative accuracy next to x = 1; ln2 is split into a high
// part with trailing zero bits (e ln2_hi exact for |e| < 2^11) and a low part.
// About 38 VALU issue slots on gfx950 against 97 for the library log, within
// 2 ulp of the correctly rounded result (checked against the host libm over
// the whole exponent range by the test-suite).
// Only finite x > 0 take the series; anything else falls back to log().
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define VSH_HD __host__ __device__
#else
#define VSH_HD
#endif

namespace vsh {

// p * s2 + c for the series: on the device as v_fma_f64 with c (a literal)
// in a scalar register pair; left to the compiler, each addend would be
// copied into a vector register pair (two VALU moves) for v_fmac_f64.  The
// same fused operation either way, so host and device agree bit for bit.
VSH_HD inline double fma_addend(double p, double s2, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(s2), "s"(c));
  return r;
#else
  return fma(p, s2, c);
#endif
}

// the series part, for finite x > 0
VSH_HD inline double log_series(double x) {
  int e;
  double m = frexp(x, &e);  // m in [0.5, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = fma_addend(1.0 / 21.0, s2, 1.0 / 19.0);
  p = fma_addend(p, s2, 1.0 / 17.0);
  p = fma_addend(p, s2, 1.0 / 15.0);
  p = fma_addend(p, s2, 1.0 / 13.0);
  p = fma_addend(p, s2, 1.0 / 11.0);
  p = fma_addend(p, s2, 1.0 / 9.0);
  p = fma_addend(p, s2, 1.0 / 7.0);
  p = fma_addend(p, s2, 1.0 / 5.0);
  p = fma_addend(p, s2, 1.0 / 3.0);
  const double two_s = 2.0 * s;
  const double lnm = fma(two_s * s2, p, two_s);
  const double ln2_hi = 6.93147180369123816490e-01;  // high bits of ln 2 (trailing zeros)
  const double ln2_lo = 1.90821492927058770002e-10;  // ln 2 - ln2_hi
  const double de = (double)e;
  return fma(de, ln2_hi, fma(de, ln2_lo, lnm));
}

VSH_HD inline double log_fast(double x) {
  if (!(x > 0.0) || !(x < INFINITY)) return log(x);
  return log_series(x);
}

}  // namespace vsh
