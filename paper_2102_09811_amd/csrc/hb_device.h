// Device-side numerical helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace hb {

template <int N>
__device__ __forceinline__ float hornerf(const float *__restrict__ c, float x) {
  float r = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) r = fmaf(r, x, c[i]);
  return r;
}

template <int N>
__device__ __forceinline__ double horner(const double *__restrict__ c, double x) {
  double r = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) r = fma(r, x, c[i]);
  return r;
}

// e^{-w} for w >= 0: Cody-Waite reduction w = k ln2 - r with the ln2 split of fdlibm, the degree-12
// Taylor polynomial of e^r on |r| <= ln2/2 (truncation < 2e-16 relative), then 2^k by ldexp, which
// also underflows gracefully; inputs are clamped at 1000 where the result is 0.  Max relative error
// about 1.5 ulp, and no range branches or selects.
__device__ __forceinline__ double exp_neg(double w) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  const double t = -fmin(w, 1000.0);
  const double k = rint(t * kLog2e);
  double r = fma(k, -kLn2Hi, t);
  r = fma(k, -kLn2Lo, r);
  double q = 1.0 / 479001600.0;
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

}  // namespace hb
