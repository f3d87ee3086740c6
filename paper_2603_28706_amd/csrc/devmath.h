// FP64 elementary functions of the action kernels (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace pns {

// FP64 elementary functions for the tangent scalars, specialised to the
// arguments that occur here (finite, positive, normal D2; |exponent argument|
// well below the overflow range), without the special-case handling of the
// general library routines.
// 1/d: hardware reciprocal seed refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  return r;
}
// 1/sqrt(a), a > 0: hardware seed refined by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double a) {
  double r = __builtin_amdgcn_rsq(a);
  r = r * fma(-0.5 * a * r, r, 1.5);
  r = r * fma(-0.5 * a * r, r, 1.5);
  return r;
}
// log(x), x > 0 normal: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.172, series to s^21.
__device__ __forceinline__ double log_pos(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;
  const double sv = f * rcp_nr(2.0 + f);
  const double s2 = sv * sv;
  double q = 2.0 / 21.0;
  q = fma(q, s2, 2.0 / 19.0);
  q = fma(q, s2, 2.0 / 17.0);
  q = fma(q, s2, 2.0 / 15.0);
  q = fma(q, s2, 2.0 / 13.0);
  q = fma(q, s2, 2.0 / 11.0);
  q = fma(q, s2, 2.0 / 9.0);
  q = fma(q, s2, 2.0 / 7.0);
  q = fma(q, s2, 2.0 / 5.0);
  q = fma(q, s2, 2.0 / 3.0);
  const double lm = fma(sv * s2, q, 2.0 * sv);
  const double de = (double)e;
  return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, lm));
}
// exp(y), |y| < 700: Cody-Waite reduction y = k ln2 + r, |r| <= ln2/2, Taylor
// polynomial of degree 13 for exp(r), scaled by 2^k.
__device__ __forceinline__ double exp_small(double y) {
  const double k = rint(y * 1.44269504088896340736);
  double r = fma(-k, 6.93147180369123816490e-01, y);
  r = fma(-k, 1.90821492927058770002e-10, r);
  double q = 1.0 / 6227020800.0;
  q = fma(q, r, 1.0 / 479001600.0);
  q = fma(q, r, 1.0 / 39916800.0);
  q = fma(q, r, 1.0 / 3628800.0);
  q = fma(q, r, 1.0 / 362880.0);
  q = fma(q, r, 1.0 / 40320.0);
  q = fma(q, r, 1.0 / 5040.0);
  q = fma(q, r, 1.0 / 720.0);
  q = fma(q, r, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return ldexp(q, (int)k);
}

}  // namespace pns
