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

// 2^{-j/64}, j = 0 .. 63, each the correctly rounded double (hex literals, from 60-digit decimal
// arithmetic).
static __constant__ double kExp2Tab[64] = {
    0x1.0000000000000p+0, 0x1.fa7c1819e90d8p-1, 0x1.f50765b6e4540p-1, 0x1.efa1bee615a27p-1,
    0x1.ea4afa2a490dap-1, 0x1.e502ee78b3ff6p-1, 0x1.dfc97337b9b5fp-1, 0x1.da9e603db3285p-1,
    0x1.d5818dcfba487p-1, 0x1.d072d4a07897cp-1, 0x1.cb720dcef9069p-1, 0x1.c67f12e57d14bp-1,
    0x1.c199bdd85529cp-1, 0x1.bcc1e904bc1d2p-1, 0x1.b7f76f2fb5e47p-1, 0x1.b33a2b84f15fbp-1,
    0x1.ae89f995ad3adp-1, 0x1.a9e6b5579fdbfp-1, 0x1.a5503b23e255dp-1, 0x1.a0c667b5de565p-1,
    0x1.9c49182a3f090p-1, 0x1.97d829fde4e50p-1, 0x1.93737b0cdc5e5p-1, 0x1.8f1ae99157736p-1,
    0x1.8ace5422aa0dbp-1, 0x1.868d99b4492edp-1, 0x1.82589994cce13p-1, 0x1.7e2f336cf4e62p-1,
    0x1.7a11473eb0187p-1, 0x1.75feb564267c9p-1, 0x1.71f75e8ec5f74p-1, 0x1.6dfb23c651a2fp-1,
    0x1.6a09e667f3bcdp-1, 0x1.6623882552225p-1, 0x1.6247eb03a5585p-1, 0x1.5e76f15ad2148p-1,
    0x1.5ab07dd485429p-1, 0x1.56f4736b527dap-1, 0x1.5342b569d4f82p-1, 0x1.4f9b2769d2ca7p-1,
    0x1.4bfdad5362a27p-1, 0x1.486a2b5c13cd0p-1, 0x1.44e086061892dp-1, 0x1.4160a21f72e2ap-1,
    0x1.3dea64c123422p-1, 0x1.3a7db34e59ff7p-1, 0x1.371a7373aa9cbp-1, 0x1.33c08b26416ffp-1,
    0x1.306fe0a31b715p-1, 0x1.2d285a6e4030bp-1, 0x1.29e9df51fdee1p-1, 0x1.26b4565e27cddp-1,
    0x1.2387a6e756238p-1, 0x1.2063b88628cd6p-1, 0x1.1d4873168b9aap-1, 0x1.1a35beb6fcb75p-1,
    0x1.172b83c7d517bp-1, 0x1.1429aaea92de0p-1, 0x1.11301d0125b51p-1, 0x1.0e3ec32d3d1a2p-1,
    0x1.0b5586cf9890fp-1, 0x1.0874518759bc8p-1, 0x1.059b0d3158574p-1, 0x1.02c9a3e778061p-1,
};

// Copy of kExp2Tab in the calling workgroup's LDS (64 doubles; the caller synchronises).
__device__ __forceinline__ void stage_exp_tab(double *etab) {
  for (int i = threadIdx.x; i < 64; i += blockDim.x) etab[i] = kExp2Tab[i];
}

// e^{-w} for w >= 0 with the table etab = 2^{-j/64} in LDS: w = k ln2 / 64 + r (the fdlibm ln2
// split scaled by 1/64, |r| <= ln2 / 128), e^{-w} = 2^{-(k >> 6)} 2^{-(k & 63)/64} e^{-r} with the
// degree-5 Taylor polynomial of e^{-r} (truncation below 4e-17 relative); inputs are clamped at 1000
// where the result is 0.  13 double operations instead of the 19 of exp_neg.
__device__ __forceinline__ double exp_neg_t(double w, const double *__restrict__ etab) {
  constexpr double k64Log2e = 92.332482616893658;  // 64 / ln 2
  constexpr double kLn2Hi64 = 6.93147180369123816490e-01 / 64;
  constexpr double kLn2Lo64 = 1.90821492927058770002e-10 / 64;
  const double x = fmin(w, 1000.0);
  const double k = rint(x * k64Log2e);
  double r = fma(k, -kLn2Hi64, x);
  r = fma(k, -kLn2Lo64, r);
  const int ki = (int)k;
  double q = -1.0 / 120.0;
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, -1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, -1.0);
  q = fma(q, r, 1.0);
  return ldexp(etab[ki & 63] * q, -(ki >> 6));
}

// Copy of 2^{+j/64}, j = 0 .. 63, in the calling workgroup's LDS: 1 and 2 kExp2Tab[64 - j] (exact
// doublings of the correctly rounded 2^{-(64-j)/64}).  The caller synchronises.
__device__ __forceinline__ void stage_exp_tab_pos(double *etab) {
  for (int i = threadIdx.x; i < 64; i += blockDim.x) etab[i] = i == 0 ? 1.0 : 2.0 * kExp2Tab[64 - i];
}

// e^{-w} for w >= 0 with etab = 2^{j/64} in LDS: k = round(-64 w / ln 2) is read from the low word
// of t = -64 w / ln 2 + 1.5 2^52 (round to nearest, exact while |k| < 2^51), r = w + k ln2 / 64
// (the fdlibm ln2 split scaled by 1/64, |r| <= ln2 / 128), and
// e^{-w} = 2^{k >> 6} 2^{(k & 63)/64} e^{-r} with the degree-5 Taylor polynomial of e^{-r}
// (truncation below 4e-17 relative); inputs are clamped at 1000 where the result is 0.
__device__ __forceinline__ double exp_neg_m(double w, const double *__restrict__ etab) {
  constexpr double kNeg64Log2e = -92.332482616893658;  // -64 / ln 2
  constexpr double kShift = 6755399441055744.0;         // 1.5 * 2^52
  constexpr double kLn2Hi64 = 6.93147180369123816490e-01 / 64;
  constexpr double kLn2Lo64 = 1.90821492927058770002e-10 / 64;
  const double x = fmin(w, 1000.0);
  const double t = fma(x, kNeg64Log2e, kShift);
  const double k = t - kShift;
  const int ki = __double2loint(t);
  double r = fma(k, kLn2Hi64, x);
  r = fma(k, kLn2Lo64, r);
  double q = -1.0 / 120.0;
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, -1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, -1.0);
  q = fma(q, r, 1.0);
  return ldexp(etab[ki & 63] * q, ki >> 6);
}

// P(x) and P'(x) of the polynomial c[0] + c[1] x + ... + c[N-1] x^{N-1}, one Horner sweep.
template <int N>
__device__ __forceinline__ void horner_d(const double *__restrict__ c, double x, double &p,
                                         double &dp) {
  p = c[N - 1];
  dp = p;
  p = fma(p, x, c[N - 2]);
#pragma unroll
  for (int i = N - 3; i >= 0; --i) {
    dp = fma(dp, x, p);
    p = fma(p, x, c[i]);
  }
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) in turn.  This renumbers them so that
// each XCD takes a contiguous range of blocks (a bijection of [0, gridDim.x)): neighbouring tasks
// then write neighbouring addresses through the same L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, r = nb & 7, x = b & 7, s = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

}  // namespace hb
