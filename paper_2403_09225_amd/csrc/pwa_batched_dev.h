// Device helpers shared by the batched-path sources (FP64/FP32/16-bit
// formats and the sliced FP16 format).
#pragma once

#include <math.h>

#include "pwa_batched.h"

namespace pwa {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void dd_add_b(double& hi, double& lo, double bhi, double blo) {
  const double s = hi + bhi;
  const double bb = s - hi;
  double e = (hi - (s - bb)) + (bhi - bb);
  e += lo + blo;
  hi = s + e;
  lo = e - (hi - s);
}

__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// ln of m in [1/16, 1) in single precision: m = f 2^e with f in
// [sqrt(1/2), sqrt(2)); ln f = 2 atanh(y) by its series through y^9
// (|y| <= 0.1716, truncation < 3e-9 relative); e ln 2 added in FP64.
__device__ __forceinline__ double ln_small(float m) {
  int e;
  float f = frexpf(m, &e);
  const bool lo = f < 0.70710678f;
  f = lo ? 2.0f * f : f;
  e = lo ? e - 1 : e;
  // y = (f - 1)/(f + 1): hardware reciprocal, then one correction of the
  // quotient from its exact residual (a Newton step on the reciprocal alone
  // leaves a one-signed error that would bias the log sum).
  const float fp1 = f + 1.0f, fm1 = f - 1.0f;
  const float r = __builtin_amdgcn_rcpf(fp1);
  const float y0 = fm1 * r;
  const float y = fmaf(fmaf(-y0, fp1, fm1), r, y0);
  const float y2 = y * y;
  float p = fmaf(y2, 1.0f / 9.0f, 1.0f / 7.0f);
  p = fmaf(p, y2, 1.0f / 5.0f);
  p = fmaf(p, y2, 1.0f / 3.0f);
  const float s = fmaf(2.0f * y * y2, p, 2.0f * y);
  return fma((double)e, 0.69314718055994530942, (double)s);
}

// ln of m in [1/16, 1) in double precision (FP64 and sliced formats): same series
// through y^21.
__device__ __forceinline__ double ln_small64(double m) {
  int e;
  double f = frexp(m, &e);
  const bool lo = f < 0.70710678118654752440;
  f = lo ? 2.0 * f : f;
  e = lo ? e - 1 : e;
  const double y = (f - 1.0) * rcp64(f + 1.0);
  const double y2 = y * y;
  double p = 1.0 / 21.0;
  p = fma(p, y2, 1.0 / 19.0);
  p = fma(p, y2, 1.0 / 17.0);
  p = fma(p, y2, 1.0 / 15.0);
  p = fma(p, y2, 1.0 / 13.0);
  p = fma(p, y2, 1.0 / 11.0);
  p = fma(p, y2, 1.0 / 9.0);
  p = fma(p, y2, 1.0 / 7.0);
  p = fma(p, y2, 1.0 / 5.0);
  p = fma(p, y2, 1.0 / 3.0);
  const double t = 2.0 * y;
  const double de = (double)e;
  return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, fma(t * y2, p, t)));
}

__device__ __forceinline__ void frozen_amp(const double* __restrict__ planes, int64_t stride,
                                           int64_t i, const double* __restrict__ tbl,
                                           const int* __restrict__ itbl, int k, int gen,
                                           double& re, double& im) {
  const double* t = tbl + k * TS;
  const double s = planes[(int64_t)itbl[k * ITS + 0] * stride + i];
  const double u = planes[(int64_t)itbl[k * ITS + 1] * stride + i] * t[TB_UMUL] + t[TB_UADD];
  const double g = planes[(int64_t)itbl[k * ITS + 2] * stride + i];
  // Flatte resonances (general path): complex width factor g + i h
  const double h = gen ? planes[(int64_t)itbl[k * ITS + IT_H] * stride + i] : 0.0;
  const double Dr = t[TB_M2] - s - t[TB_NGE] * h, Di = t[TB_NGE] * g;
  const double bu = t[TB_BETA] * u * rcp64(Dr * Dr + Di * Di);
  re = bu * Dr;
  im = -bu * Di;
}

// ------------------------------------------------------------------------
// Sliced FP16 format.  A value x with |x| < 2^E is cut as
//   x 2^(9-E) = q0 + 2^-9 q1 + 2^-18 q2 + 2^-27 q3 + r,   |r| <= 2^-28,
// q_s = nearest integer of the running remainder (times 2^9 per slice):
// |q0| <= 512, |q1..q3| <= 256, all exact in FP16.  The subtraction of an
// integer from the remainder and the power-of-two steps are exact in FP64.
// ------------------------------------------------------------------------
__device__ __forceinline__ void slice4(double x, _Float16* q, int64_t plane) {
#pragma unroll
  for (int s = 0; s < kSlices; ++s) {
    const double r = rint(x);
    q[s * plane] = (_Float16)r;
    x = (x - r) * 512.0;
  }
}

// Exponent E of the largest magnitude (|m| < 2^E); 0 for a zero or
// non-finite maximum.
__device__ __forceinline__ int max_exponent(double m) {
  int e = 0;
  if (m > 0.0 && isfinite(m)) frexp(m, &e);
  return e;
}

// Exponent G_b of start b's largest real or imaginary coupling component.
__device__ __forceinline__ int coupling_exponent(const double* __restrict__ C, int K, int b) {
  double m = 0.0;
  for (int k = 0; k < K; ++k) m = fmax(m, fmax(fabs(C[2 * (b * K + k)]), fabs(C[2 * (b * K + k) + 1])));
  return max_exponent(m);
}

}  // namespace pwa
