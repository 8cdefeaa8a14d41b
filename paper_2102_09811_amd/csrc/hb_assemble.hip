// Assembly of the block-Toeplitz single-layer (V_h^d, p0 x p0) and double-layer (K_h^d, p0 x p1)
// matrices for every temporal distance d (Sec. 3.1, 3.2, 5).
//
// Temporal part, per point pair r = x - y (rho = |r|, rn = r . n_y):
//   blocks d < D (D = d_switch): second differences of G^{dtau dt}(rho, i h) and of its normal
//     derivative over the levels i = 0..D (the paper's reuse of one evaluation per delta = i h,
//     Sec. 5.1 / Tables 5.1-5.2), plus the h G^{dtau}(rho, 0) term of block 0;
//       F(rho, delta)           = rho A(z) / (8 pi alpha^2),    z = rho / (2 sqrt(alpha delta))
//       alpha dF/dn_y (r, delta) = -(rn / rho) B(z) / (8 pi alpha),
//       A = (1 + 1/(2z^2)) erf z + e^{-z^2}/(z sqrt pi),  B = (1 - 1/(2z^2)) erf z + e^{-z^2}/(z sqrt pi)
//     (Sec. 3.1 eq. for G^{dtau dt}, Sec. 3.2 eq. for alpha dG^{dtau dt}/dn), with the exact small-z
//     series of A and B for z < 1/2 (B cancels like 1/z^2 in closed form);
//   blocks d >= D: the even Taylor series of the hat-weighted kernel (exact rewriting of the same
//     time integral, no second difference): h^2 G(rho, d h) P_d(w) and h^2 alpha dG/dn(r, d h)
//     P^K_d(w) with w = rho^2 / (4 alpha d h) and tabulated polynomials P_d, P^K_d.
// Spatial part: Radon's 7-point rule on both panels for separated pairs (k_separated), regularised
// [0,1]^4 rules for touching pairs (k_touching).  V entries are stored by their single owner; K
// contributions are added to the three trial vertices with atomics.
#include "hb_internal.h"

namespace hb {
namespace {

constexpr double kInvSqrtPi = 0.56418958354775628695;
constexpr double kFourInvSqrtPi = 2.2567583341910251478;

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

// One closed-form level: rA = rho A(z), kB = B(z) / rho.
__device__ __forceinline__ void closed_level(const AsmParams &p, int i, double rho,
                                             double inv_rho, double &rA, double &kB) {
  const double c = p.lv.c[i];
  const double z = rho * c;
  if (z < 0.5) {
    const double z2 = z * z;
    const double sa = horner<kSeriesN>(p.serA, z2);
    const double sb = horner<kSeriesN>(p.serB, z2);
    rA = fma(rho * z * kInvSqrtPi, sa, p.lv.t2[i]);
    kB = kFourInvSqrtPi * c * sb;
  } else {
    const double e = exp(-z * z);
    const double er = erf(z);
    const double es = er * p.lv.s2[i] * inv_rho;   // erf * 2 alpha delta / rho
    const double ps = e * p.lv.s1[i];              // e^{-z^2} 2 sqrt(alpha delta)/sqrt(pi)
    rA = fma(rho, er, es) + ps;
    kB = inv_rho * (er + (ps - es) * inv_rho);
  }
}

template <typename TS>
__device__ __forceinline__ void store_block(const AsmParams &p, int d, int l, int m, double v) {
  TS *V = (TS *)p.V;
  V[((size_t)d * p.ne + l) * p.ne + m] = (TS)v;
}

template <typename TS>
__device__ __forceinline__ void add_block_K(const AsmParams &p, int d, int l, int j, double v) {
  TS *K = (TS *)p.K;
  atomicAdd(&K[((size_t)d * p.ne + l) * p.nv + j], (TS)v);
}

constexpr int kLC = 2;  // closed-form levels per pass over the quadrature points
constexpr int kLT = 1;  // Taylor blocks per pass over the quadrature points

// Level sums of one pass: S[0], S[1] carry levels i0-2, i0-1; S[2 + j] is level i0 + j.
struct LevelSums {
  double V[kLC + 2];
  double K[kLC + 2][3];
};

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

// Emit the blocks completed by the pass over levels i0 .. i0+kLC-1 (clipped to D).
template <typename TS, int D>
__device__ __forceinline__ void emit_pass(const AsmParams &p, int i0, int l, int m,
                                          const int vtx[3], double scale, const LevelSums &S,
                                          double sV, const double sK[3]) {
  const int i1 = min(i0 + kLC - 1, D);
#pragma unroll
  for (int j = 0; j < kLC + 1; ++j) {
    const int d = i0 - 1 + j;              // blocks i0-1 .. i1-1
    if (d < 0 || d > i1 - 1 || d >= D || d >= p.nt) continue;
    const int c = d - i0 + 2;              // slot of level d
    double v, k[3];
    if (d == 0) {
      v = p.kVs * sV + p.kV * (S.V[c] - S.V[c + 1]);
#pragma unroll
      for (int q = 0; q < 3; ++q) k[q] = p.kKs * sK[q] + p.kK * (S.K[c + 1][q] - S.K[c][q]);
    } else {
      v = p.kV * (2.0 * S.V[c] - S.V[c + 1] - S.V[c - 1]);
#pragma unroll
      for (int q = 0; q < 3; ++q) k[q] = -p.kK * (2.0 * S.K[c][q] - S.K[c + 1][q] - S.K[c - 1][q]);
    }
    if (p.do_V) store_block<TS>(p, d, l, m, v * scale);
    if (p.do_K) {
#pragma unroll
      for (int q = 0; q < 3; ++q) add_block_K<TS>(p, d, l, vtx[q], k[q] * scale);
    }
  }
}

__device__ __forceinline__ void shift_carry(LevelSums &S) {
  S.V[0] = S.V[kLC];
  S.V[1] = S.V[kLC + 1];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    S.K[0][q] = S.K[kLC][q];
    S.K[1][q] = S.K[kLC + 1][q];
  }
#pragma unroll
  for (int j = 2; j < kLC + 2; ++j) S.V[j] = S.K[j][0] = S.K[j][1] = S.K[j][2] = 0.0;
}

// One pass of the separated kernel over the 49 point pairs for closed-form levels I0..I0+kLC-1,
// then the blocks it completes; recurses to the next pass at compile time.
template <typename TS, int D, int I0>
__device__ __forceinline__ void separated_pass(const AsmParams &p, int l, int m, const int vtx[3],
                                               bool touch, double n0, double n1, double n2,
                                               double scale, double shift, const double *xg,
                                               LevelSums &S, double &sV, double sK[3]) {
  if constexpr (I0 <= D) {
    const int ne = p.ne;
#pragma unroll 1
    for (int b = 0; b < kFarN; ++b) {
      const double y0 = p.geom[(b * 3 + 0) * ne + m] + shift;
      const double y1 = p.geom[(b * 3 + 1) * ne + m];
      const double y2 = p.geom[(b * 3 + 2) * ne + m];
      const double wb = p.w7[b];
      double tK[kLC], tsK = 0.0;
#pragma unroll
      for (int j = 0; j < kLC; ++j) tK[j] = 0.0;
#pragma unroll 1
      for (int a = 0; a < kFarN; ++a) {
        const double rx = xg[(a * 3 + 0) * ne] - y0;
        const double ry = xg[(a * 3 + 1) * ne] - y1;
        const double rz = xg[(a * 3 + 2) * ne] - y2;
        const double rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double rho = sqrt(rho2);
        const double inv_rho = 1.0 / rho;
        const double wa = p.w7[a];
        const double W = wa * wb;
        const double wrn = wa * fma(rx, n0, fma(ry, n1, rz * n2));
        if constexpr (I0 == 0) {
          sV = fma(W, inv_rho, sV);
          tsK = fma(wrn, inv_rho * inv_rho * inv_rho, tsK);
        }
#pragma unroll
        for (int j = 0; j < kLC; ++j) {
          if (I0 + j > D) continue;
          double rA, kB;
          level_terms(p, I0 + j, rho, inv_rho, rA, kB);
          S.V[2 + j] = fma(W, rA, S.V[2 + j]);
          tK[j] = fma(wrn, kB, tK[j]);
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double phi = wb * p.lam7[b][k];
#pragma unroll
        for (int j = 0; j < kLC; ++j) S.K[2 + j][k] = fma(phi, tK[j], S.K[2 + j][k]);
        if constexpr (I0 == 0) sK[k] = fma(phi, tsK, sK[k]);
      }
    }
    if (!touch) emit_pass<TS, D>(p, I0, l, m, vtx, scale, S, sV, sK);
    shift_carry(S);
    separated_pass<TS, D, I0 + kLC>(p, l, m, vtx, touch, n0, n1, n2, scale, shift, xg, S, sV, sK);
  }
}

// ------------------------------------------------------------------------------------------
// Separated pairs: workgroup = (test panel l, 256 consecutive trial panels m); lane = m.
// ------------------------------------------------------------------------------------------
template <typename TS, int D, bool MIXED>
__global__ __launch_bounds__(256, 2) void k_separated(const AsmParams *__restrict__ pp) {
  const AsmParams &p = *pp;
  const int l = blockIdx.y;
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= p.ne) return;
  const int ne = p.ne;
  const int32_t *tl = p.tris + 3 * l;
  const int vtx[3] = {p.tris[3 * m], p.tris[3 * m + 1], p.tris[3 * m + 2]};
  bool touch = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) touch |= tl[i] == vtx[j];
  const double n0 = p.geom[21 * ne + m], n1 = p.geom[22 * ne + m], n2 = p.geom[23 * ne + m];
  const double scale = p.geom[24 * ne + l] * p.geom[24 * ne + m];
  // touching lanes integrate a far-away copy of their panel and store nothing
  const double shift = touch ? 1.0e3 : 0.0;
  const double *xg = p.geom + l;  // test nodes: xg[(a*3+c)*ne]

  // ---- closed-form levels 0 .. D, kLC per pass ----
  LevelSums S;
#pragma unroll
  for (int j = 0; j < kLC + 2; ++j) S.V[j] = S.K[j][0] = S.K[j][1] = S.K[j][2] = 0.0;
  double sV = 0.0, sK[3] = {0.0, 0.0, 0.0};
  separated_pass<TS, D, 0>(p, l, m, vtx, touch, n0, n1, n2, scale, shift, xg, S, sV, sK);

  // ---- Taylor blocks d = D .. nt-1, kLT at a time ----
  for (int d0 = D; d0 < p.nt; d0 += kLT) {
    double TV[kLT], TK[kLT][3];
#pragma unroll
    for (int j = 0; j < kLT; ++j) TV[j] = TK[j][0] = TK[j][1] = TK[j][2] = 0.0;
#pragma unroll 1
    for (int b = 0; b < kFarN; ++b) {
      const double y0 = p.geom[(b * 3 + 0) * ne + m] + shift;
      const double y1 = p.geom[(b * 3 + 1) * ne + m];
      const double y2 = p.geom[(b * 3 + 2) * ne + m];
      const double wb = p.w7[b];
      double tk[kLT];
#pragma unroll
      for (int j = 0; j < kLT; ++j) tk[j] = 0.0;
#pragma unroll 1
      for (int a = 0; a < kFarN; ++a) {
        const double rx = xg[(a * 3 + 0) * ne] - y0;
        const double ry = xg[(a * 3 + 1) * ne] - y1;
        const double rz = xg[(a * 3 + 2) * ne] - y2;
        const double rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double wa = p.w7[a];
        const double W = wa * wb;
        const double wrn = wa * fma(rx, n0, fma(ry, n1, rz * n2));
        if (MIXED && d0 >= p.mixed_d_min) {
          // mixed precision: the kernel value and its polynomial in float (hardware exp,
          // degree-8 series), the accumulation in double
#pragma unroll
          for (int j = 0; j < kLT; ++j) {
            const int d = min(d0 + j, p.nt - 1);
            const float w = (float)(rho2 * p.tscale[3 * d + 2]);
            const float e = __expf(-w);
            const float pv = hornerf<kTaylorN32>(p.taylor32 + (size_t)(2 * d) * kTaylorN32, w);
            const float pk = hornerf<kTaylorN32>(p.taylor32 + (size_t)(2 * d + 1) * kTaylorN32, w);
            TV[j] += W * (double)(e * pv);
            tk[j] += wrn * (double)(e * pk);
          }
        } else {
#pragma unroll
          for (int j = 0; j < kLT; ++j) {
            const int d = min(d0 + j, p.nt - 1);
            const double w = rho2 * p.tscale[3 * d + 2];
            const double e = exp(-w);
            const double pv = horner<kTaylorN>(p.taylor + (size_t)(2 * d) * kTaylorN, w);
            const double pk = horner<kTaylorN>(p.taylor + (size_t)(2 * d + 1) * kTaylorN, w);
            TV[j] = fma(W * e, pv, TV[j]);
            tk[j] = fma(wrn * e, pk, tk[j]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double phi = wb * p.lam7[b][k];
#pragma unroll
        for (int j = 0; j < kLT; ++j) TK[j][k] = fma(phi, tk[j], TK[j][k]);
      }
    }
    if (!touch) {
#pragma unroll
      for (int j = 0; j < kLT; ++j) {
        const int d = d0 + j;
        if (d >= p.nt) continue;
        if (p.do_V) store_block<TS>(p, d, l, m, TV[j] * p.tscale[3 * d] * scale);
        if (p.do_K) {
          const double ks = p.tscale[3 * d + 1] * scale;
#pragma unroll
          for (int k = 0; k < 3; ++k) add_block_K<TS>(p, d, l, vtx[k], TK[j][k] * ks);
        }
      }
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------------------------------
// Touching pairs: one wave per ordered pair; lanes stride over the regularised rule's points.
// ------------------------------------------------------------------------------------------
struct TouchPoint {
  double rho2, rho, inv_rho, W, wrn, l0, l1, l2;
};

__device__ __forceinline__ TouchPoint touch_point(const TouchPair &tp, const double *__restrict__ tab,
                                                  int ntab, int q, bool need_rho) {
  const double a1 = tab[q], a2 = tab[ntab + q], a3 = tab[2 * ntab + q], a4 = tab[3 * ntab + q];
  const double rx = a1 * tp.E1[0] + a2 * tp.E2[0] + a3 * tp.F1[0] + a4 * tp.F2[0];
  const double ry = a1 * tp.E1[1] + a2 * tp.E2[1] + a3 * tp.F1[1] + a4 * tp.F2[1];
  const double rz = a1 * tp.E1[2] + a2 * tp.E2[2] + a3 * tp.F1[2] + a4 * tp.F2[2];
  TouchPoint t;
  t.rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
  if (need_rho) {
    t.rho = sqrt(t.rho2);
    t.inv_rho = 1.0 / t.rho;
  } else {
    t.rho = t.inv_rho = 0.0;
  }
  t.W = tab[4 * ntab + q];
  t.wrn = t.W * fma(rx, tp.n[0], fma(ry, tp.n[1], rz * tp.n[2]));
  t.l0 = tab[5 * ntab + q];
  t.l1 = tab[6 * ntab + q];
  t.l2 = tab[7 * ntab + q];
  return t;
}

template <typename TS, int D, int I0>
__device__ __forceinline__ void touching_pass(const AsmParams &p, const TouchPair &tp,
                                              const double *__restrict__ tab, int ntab, int lane,
                                              int l, int m, const int vtx[3], LevelSums &S,
                                              double &sV, double sK[3]) {
  if constexpr (I0 <= D) {
#pragma unroll 1
    for (int q = lane; q < ntab; q += 64) {
      const TouchPoint t = touch_point(tp, tab, ntab, q, true);
      if constexpr (I0 == 0) {
        sV = fma(t.W, t.inv_rho, sV);
        const double u = t.wrn * t.inv_rho * t.inv_rho * t.inv_rho;
        sK[0] = fma(u, t.l0, sK[0]);
        sK[1] = fma(u, t.l1, sK[1]);
        sK[2] = fma(u, t.l2, sK[2]);
      }
#pragma unroll
      for (int j = 0; j < kLC; ++j) {
        if (I0 + j > D) continue;
        double rA, kB;
        level_terms(p, I0 + j, t.rho, t.inv_rho, rA, kB);
        S.V[2 + j] = fma(t.W, rA, S.V[2 + j]);
        const double u = t.wrn * kB;
        S.K[2 + j][0] = fma(u, t.l0, S.K[2 + j][0]);
        S.K[2 + j][1] = fma(u, t.l1, S.K[2 + j][1]);
        S.K[2 + j][2] = fma(u, t.l2, S.K[2 + j][2]);
      }
    }
#pragma unroll
    for (int j = 2; j < kLC + 2; ++j) {
      S.V[j] = wave_sum(S.V[j]);
#pragma unroll
      for (int k = 0; k < 3; ++k) S.K[j][k] = wave_sum(S.K[j][k]);
    }
    if constexpr (I0 == 0) {
      sV = wave_sum(sV);
#pragma unroll
      for (int k = 0; k < 3; ++k) sK[k] = wave_sum(sK[k]);
    }
    if (lane == 0) emit_pass<TS, D>(p, I0, l, m, vtx, tp.scale, S, sV, sK);
    shift_carry(S);
    touching_pass<TS, D, I0 + kLC>(p, tp, tab, ntab, lane, l, m, vtx, S, sV, sK);
  }
}

template <typename TS, int D>
__global__ __launch_bounds__(64, 2) void k_touching(const AsmParams *__restrict__ pp,
                                                    const TouchPair *__restrict__ pairs,
                                                    const double *__restrict__ tab, int ntab) {
  const AsmParams &p = *pp;
  const TouchPair &tp = pairs[blockIdx.x];
  const int lane = threadIdx.x;
  const int l = tp.l, m = tp.m;
  const int vtx[3] = {tp.vtx[0], tp.vtx[1], tp.vtx[2]};

  LevelSums S;
#pragma unroll
  for (int j = 0; j < kLC + 2; ++j) S.V[j] = S.K[j][0] = S.K[j][1] = S.K[j][2] = 0.0;
  double sV = 0.0, sK[3] = {0.0, 0.0, 0.0};
  touching_pass<TS, D, 0>(p, tp, tab, ntab, lane, l, m, vtx, S, sV, sK);

  for (int d0 = D; d0 < p.nt; d0 += kLT) {
    double TV[kLT], TK[kLT][3];
#pragma unroll
    for (int j = 0; j < kLT; ++j) TV[j] = TK[j][0] = TK[j][1] = TK[j][2] = 0.0;
#pragma unroll 1
    for (int q = lane; q < ntab; q += 64) {
      const TouchPoint t = touch_point(tp, tab, ntab, q, false);
#pragma unroll
      for (int j = 0; j < kLT; ++j) {
        const int d = min(d0 + j, p.nt - 1);
        const double w = t.rho2 * p.tscale[3 * d + 2];
        const double e = exp(-w);
        const double pv = horner<kTaylorN>(p.taylor + (size_t)(2 * d) * kTaylorN, w);
        const double pk = horner<kTaylorN>(p.taylor + (size_t)(2 * d + 1) * kTaylorN, w);
        TV[j] = fma(t.W * e, pv, TV[j]);
        const double u = t.wrn * e * pk;
        TK[j][0] = fma(u, t.l0, TK[j][0]);
        TK[j][1] = fma(u, t.l1, TK[j][1]);
        TK[j][2] = fma(u, t.l2, TK[j][2]);
      }
    }
#pragma unroll
    for (int j = 0; j < kLT; ++j) {
      TV[j] = wave_sum(TV[j]);
#pragma unroll
      for (int k = 0; k < 3; ++k) TK[j][k] = wave_sum(TK[j][k]);
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < kLT; ++j) {
        const int d = d0 + j;
        if (d >= p.nt) continue;
        if (p.do_V) store_block<TS>(p, d, l, m, TV[j] * p.tscale[3 * d] * tp.scale);
        if (p.do_K) {
          const double ks = p.tscale[3 * d + 1] * tp.scale;
#pragma unroll
          for (int k = 0; k < 3; ++k) add_block_K<TS>(p, d, l, vtx[k], TK[j][k] * ks);
        }
      }
    }
  }
}

}  // namespace

template <typename TS, int D>
static void launch_sep(dim3 grid, hipStream_t s, const AsmParams *dp, bool mixed) {
  if (mixed) hipLaunchKernelGGL((k_separated<TS, D, true>), grid, dim3(256), 0, s, dp);
  else hipLaunchKernelGGL((k_separated<TS, D, false>), grid, dim3(256), 0, s, dp);
}

void launch_assemble_separated(const AsmParams *dp, const AsmParams &p, int precision,
                               int storage_f32, hipStream_t s) {
  dim3 grid((p.ne + 255) / 256, p.ne);
  const bool mixed = precision == HB_PREC_MIXED;
  if (p.dsw == 16) {
    if (storage_f32) launch_sep<float, 16>(grid, s, dp, mixed);
    else launch_sep<double, 16>(grid, s, dp, mixed);
  } else {
    if (storage_f32) launch_sep<float, 8>(grid, s, dp, mixed);
    else launch_sep<double, 8>(grid, s, dp, mixed);
  }
}

void launch_assemble_touching(const AsmParams *dp, const AsmParams &p, const TouchPair *pairs,
                              int64_t npairs, const SSRule &rule, int storage_f32, hipStream_t s) {
  dim3 grid((unsigned)npairs);
  if (p.dsw == 16) {
    if (storage_f32) hipLaunchKernelGGL((k_touching<float, 16>), grid, dim3(64), 0, s, dp, pairs, rule.d, rule.n);
    else hipLaunchKernelGGL((k_touching<double, 16>), grid, dim3(64), 0, s, dp, pairs, rule.d, rule.n);
  } else {
    if (storage_f32) hipLaunchKernelGGL((k_touching<float, 8>), grid, dim3(64), 0, s, dp, pairs, rule.d, rule.n);
    else hipLaunchKernelGGL((k_touching<double, 8>), grid, dim3(64), 0, s, dp, pairs, rule.d, rule.n);
  }
}

}  // namespace hb
