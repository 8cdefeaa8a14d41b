// Closed-form temporal terms shared by the assembly kernels: at level i (delta = i h,
// z = rho / (2 sqrt(alpha delta))) the brackets of G^{dtau dt} and of its normal derivative
// (Sec. 3.1, 3.2): rA = rho A(z), kB = B(z) / rho, with the exact small-z series below z = 1/2.
#pragma once
#include "hb_device.h"
#include "hb_internal.h"

namespace hb {

constexpr double kInvSqrtPi = 0.56418958354775628695;
constexpr double kFourInvSqrtPi = 2.2567583341910251478;

// One closed-form level at delta > 0 given its constants c = 1/(2 sqrt(alpha delta)),
// s2 = 2 alpha delta, s1 = 2 sqrt(alpha delta)/sqrt(pi), t2 = 2 s1: rA = rho A(z), kB = B(z) / rho.
__device__ __forceinline__ void closed_level_at(const AsmParams &p, double c, double s2, double s1,
                                                double t2, double rho, double inv_rho, double &rA,
                                                double &kB) {
  const double z = rho * c;
  if (z < 0.5) {
    const double z2 = z * z;
    const double sa = horner<kSeriesN>(p.serA, z2);
    const double sb = horner<kSeriesN>(p.serB, z2);
    rA = fma(rho * z * kInvSqrtPi, sa, t2);
    kB = kFourInvSqrtPi * c * sb;
  } else {
    const double e = exp_neg(z * z);
    const double er = erf(z);
    const double es = er * s2 * inv_rho;   // erf * 2 alpha delta / rho
    const double ps = e * s1;              // e^{-z^2} 2 sqrt(alpha delta)/sqrt(pi)
    rA = fma(rho, er, es) + ps;
    kB = inv_rho * (er + (ps - es) * inv_rho);
  }
}

// The same at the uniform level i (delta = i h > 0).
__device__ __forceinline__ void closed_level(const AsmParams &p, int i, double rho,
                                             double inv_rho, double &rA, double &kB) {
  closed_level_at(p, p.lv.c[i], p.lv.s2[i], p.lv.s1[i], p.lv.t2[i], rho, inv_rho, rA, kB);
}

// rho A and B / rho at level i (i = 0: the delta -> 0 limits A = B = 1).
__device__ __forceinline__ void level_terms(const AsmParams &p, int i, double rho, double inv_rho,
                                            double &rA, double &kB) {
  if (i == 0) {
    rA = rho;
    kB = inv_rho;
  } else {
    closed_level(p, i, rho, inv_rho, rA, kB);
  }
}

}  // namespace hb
