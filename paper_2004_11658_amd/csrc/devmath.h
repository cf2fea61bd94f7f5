// Device tanh for the network activations.
#pragma once
#include <hip/hip_runtime.h>

namespace dp {

// FP64 tanh from tanh|x| = 1 - 2 / (exp(2|x|) + 1):
//   exp(y) = 2^k exp(r), k = rint(y / ln 2), r = y - k ln2_hi - k ln2_lo (Cody-Waite),
//   exp(r) by its Taylor series to degree 12 (|r| <= 0.347, truncation < 2e-16),
//   1 / (e + 1) by the hardware reciprocal and two Newton steps.
// |x| is clamped at 20, where tanh rounds to 1.  Absolute error <= 3e-16 (the
// relative error of tiny results is larger; the network uses tanh values additively
// and through 1 - tanh^2, so the absolute error is what matters).
__device__ __forceinline__ double dp_tanh(double x) {
  const double ln2hi = 6.93147180369123816490e-01;
  const double ln2lo = 1.90821492927058770002e-10;
  double ax = fmin(fabs(x), 20.0);
  double y = 2.0 * ax;
  double k = __builtin_rint(y * 1.4426950408889634074);
  double r = fma(-k, ln2lo, fma(-k, ln2hi, y));
  double p = 1.0 / 479001600.0;
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  double e = __builtin_amdgcn_ldexp(p, (int)k);
  double d = e + 1.0;
  double q = __builtin_amdgcn_rcp(d);
  q = fma(q, fma(-d, q, 1.0), q);
  q = fma(q, fma(-d, q, 1.0), q);
  double t = fma(-2.0, q, 1.0);
  return copysign(t, x);
}

// FP32 tanh from the same identity with the hardware exp2 and reciprocal
// (about 1 ulp each; absolute error ~1e-7).
__device__ __forceinline__ float dp_tanh(float x) {
  float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);  // exp(2x) = 2^(2x log2 e)
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

}  // namespace dp
