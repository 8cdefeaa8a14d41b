// Near-field assembly (the paper's outlook, Sec. 6.2: with a fast multipole method the formulae of
// Sec. 3 give the near-field entries only): the blocks V_h^d[l][m] and the three p1 trial
// contributions of K_h^d for a list of ordered panel pairs, stored per pair, with the kernels and
// rules of the full assembly (closed form below d_switch, the even Taylor tables above; Radon's
// rule for separated pairs, the regularised rules for touching ones).
#include "hb_closed.h"
#include "hb_device.h"
#include "hb_internal.h"

namespace hb {
namespace {

// V^d(rho) and K^d(r) / (r . n_y) at one point pair for block d (N = 0: closed form)
template <int N>
__device__ __forceinline__ void vk_value(const AsmParams &p, double rho2, int d,
                                         const double *__restrict__ tscale,
                                         const double *__restrict__ taylor, const double *etab,
                                         double &v, double &krn) {
  if constexpr (N == 0) {
    const double rho = sqrt(rho2), inv_rho = 1.0 / rho;
    if (d == 0) {
      double rA1, kB1;
      closed_level(p, 1, rho, inv_rho, rA1, kB1);
      v = p.kVs * inv_rho + p.kV * (rho - rA1);
      krn = p.kKs * inv_rho * inv_rho * inv_rho + p.kK * (kB1 - inv_rho);
    } else {
      double rm, km, r0, k0, rp, kp;
      level_terms(p, d - 1, rho, inv_rho, rm, km);
      level_terms(p, d, rho, inv_rho, r0, k0);
      level_terms(p, d + 1, rho, inv_rho, rp, kp);
      v = p.kV * (2.0 * r0 - rp - rm);
      krn = -p.kK * (2.0 * k0 - kp - km);
    }
  } else {
    const double w = rho2 * tscale[3 * d + 2];
    const double e = exp_neg_m(w, etab);
    const double *cv = taylor + (size_t)(2 * d) * kTaylorN;
    v = tscale[3 * d] * e * horner<N>(cv, w);
    krn = tscale[3 * d + 1] * e * horner<N>(cv + kTaylorN, w);
  }
}

template <int N>
__device__ __forceinline__ void near_sep_block(const AsmParams &p, int l, int m, int d,
                                               const double *tscale, const double *taylor,
                                               const double *etab, double &V, double K[3]) {
  const int ne = p.ne;
  const double n0 = p.geom[21 * ne + m], n1 = p.geom[22 * ne + m], n2 = p.geom[23 * ne + m];
  V = 0.0;
  K[0] = K[1] = K[2] = 0.0;
#pragma unroll 1
  for (int a = 0; a < kFarN; ++a) {
    const double x0 = p.geom[(a * 3 + 0) * ne + l], x1 = p.geom[(a * 3 + 1) * ne + l],
                 x2 = p.geom[(a * 3 + 2) * ne + l];
#pragma unroll 1
    for (int b = 0; b < kFarN; ++b) {
      const double rx = x0 - p.geom[(b * 3 + 0) * ne + m];
      const double ry = x1 - p.geom[(b * 3 + 1) * ne + m];
      const double rz = x2 - p.geom[(b * 3 + 2) * ne + m];
      double v, krn;
      vk_value<N>(p, fma(rx, rx, fma(ry, ry, rz * rz)), d, tscale, taylor, etab, v, krn);
      const double W = p.w7[a] * p.w7[b];
      V = fma(W, v, V);
      const double u = W * krn * fma(rx, n0, fma(ry, n1, rz * n2));
      K[0] = fma(u, p.lam7[b][0], K[0]);
      K[1] = fma(u, p.lam7[b][1], K[1]);
      K[2] = fma(u, p.lam7[b][2], K[2]);
    }
  }
}

// Rule point q of class cls (uniform): the reference coordinates and the trial barycentrics.  The
// vertex rule stores the coordinates c = (x1, x2, -y1, -y2) themselves, so its barycentrics
// (1 - y1, y1 - y2, y2) follow from them; the identical rule's third and fourth and the edge
// rule's third coordinate are zero, and the edge rule's fourth is -y2.
__device__ __forceinline__ void rule_entries(const double *__restrict__ tab, int ntab, int cls,
                                             int q, double &a1, double &a2, double &a3, double &a4,
                                             double &b0, double &b1, double &b2) {
  a1 = tab[q];
  a2 = tab[ntab + q];
  a3 = cls == 1 ? tab[2 * ntab + q] : 0.0;
  a4 = cls == 3 ? 0.0 : tab[3 * ntab + q];
  if (cls == 1) {
    b0 = 1.0 + a3;
    b1 = a4 - a3;
    b2 = -a4;
  } else {
    b0 = tab[5 * ntab + q];
    b1 = tab[6 * ntab + q];
    b2 = cls == 2 ? -a4 : tab[7 * ntab + q];
  }
}

template <int N>
__device__ __forceinline__ void near_touch_block(const AsmParams &p, const TouchPair &tp,
                                                 const double *__restrict__ tab, int ntab, int cls,
                                                 int lane, int d, const double *tscale,
                                                 const double *taylor, const double *etab,
                                                 double &V, double K[3]) {
  V = 0.0;
  K[0] = K[1] = K[2] = 0.0;
#pragma unroll 1
  for (int q = lane; q < ntab; q += 64) {
    double a1, a2, a3, a4, b0, b1, b2;
    rule_entries(tab, ntab, cls, q, a1, a2, a3, a4, b0, b1, b2);
    const double rx = a1 * tp.E1[0] + a2 * tp.E2[0] + a3 * tp.F1[0] + a4 * tp.F2[0];
    const double ry = a1 * tp.E1[1] + a2 * tp.E2[1] + a3 * tp.F1[1] + a4 * tp.F2[1];
    const double rz = a1 * tp.E1[2] + a2 * tp.E2[2] + a3 * tp.F1[2] + a4 * tp.F2[2];
    double v, krn;
    vk_value<N>(p, fma(rx, rx, fma(ry, ry, rz * rz)), d, tscale, taylor, etab, v, krn);
    const double W = tab[4 * ntab + q];
    V = fma(W, v, V);
    const double u = W * krn * fma(rx, tp.n[0], fma(ry, tp.n[1], rz * tp.n[2]));
    K[0] = fma(u, b0, K[0]);
    K[1] = fma(u, b1, K[1]);
    K[2] = fma(u, b2, K[2]);
  }
}

// Taylor blocks d and d + 1 of one pass (the same polynomial length N) in one sweep over the rule
// points, sharing the geometry, the weights and the basis values
template <int N>
__device__ __forceinline__ void near_touch_block2(const AsmParams &p, const TouchPair &tp,
                                                  const double *__restrict__ tab, int ntab, int cls,
                                                  int lane, int d, const double *tscale,
                                                  const double *taylor, const double *etab,
                                                  double (&V)[2], double (&K)[2][3]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) V[b] = K[b][0] = K[b][1] = K[b][2] = 0.0;
#pragma unroll 1
  for (int q = lane; q < ntab; q += 64) {
    double a1, a2, a3, a4, b0, b1, b2;
    rule_entries(tab, ntab, cls, q, a1, a2, a3, a4, b0, b1, b2);
    const double rx = a1 * tp.E1[0] + a2 * tp.E2[0] + a3 * tp.F1[0] + a4 * tp.F2[0];
    const double ry = a1 * tp.E1[1] + a2 * tp.E2[1] + a3 * tp.F1[1] + a4 * tp.F2[1];
    const double rz = a1 * tp.E1[2] + a2 * tp.E2[2] + a3 * tp.F1[2] + a4 * tp.F2[2];
    const double rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const double W = tab[4 * ntab + q];
    const double rn = fma(rx, tp.n[0], fma(ry, tp.n[1], rz * tp.n[2]));
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      double v, krn;
      vk_value<N>(p, rho2, d + b, tscale, taylor, etab, v, krn);
      V[b] = fma(W, v, V[b]);
      const double u = W * krn * rn;
      K[b][0] = fma(u, b0, K[b][0]);
      K[b][1] = fma(u, b1, K[b][1]);
      K[b][2] = fma(u, b2, K[b][2]);
    }
  }
}

// Block d dispatched to the polynomial length of its pass (0: closed form; tlen: the pair class's
// distance-bounded lengths, one of kPolyLens, indexed by the first block of the pass)
#define HB_NEAR_DISPATCH(CALL)                                           \
  switch (d < p.dsw ? 0 : tlen[d - ((d - p.dsw) & 1)]) {                \
    case 0: CALL(0); break;                                              \
    case 5: CALL(5); break;                                              \
    case 6: CALL(6); break;                                              \
    case 7: CALL(7); break;                                              \
    case 8: CALL(8); break;                                              \
    case 9: CALL(9); break;                                              \
    case 10: CALL(10); break;                                            \
    case 11: CALL(11); break;                                            \
    case 13: CALL(13); break;                                            \
    case 15: CALL(15); break;                                            \
    case 17: CALL(17); break;                                            \
    case 19: CALL(19); break;                                            \
    case 21: CALL(21); break;                                            \
    case 25: CALL(25); break;                                            \
    default: CALL(29); break;                                            \
  }

// one lane per separated near pair (l, m) = sep[e] -> entry index ent[e]
__global__ __launch_bounds__(256) void k_near_separated(const AsmParams *__restrict__ pp,
                                                        const double *__restrict__ tscale,
                                                        const double *__restrict__ taylor,
                                                        const int32_t *__restrict__ tlen,
                                                        const int32_t *__restrict__ sep, int nsep,
                                                        int64_t nnz, double *__restrict__ Vn,
                                                        double *__restrict__ Kn) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  stage_exp_tab_pos(etab);
  __syncthreads();
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nsep) return;
  const int l = sep[3 * e], m = sep[3 * e + 1], ent = sep[3 * e + 2];
  const double scale = p.geom[24 * p.ne + l] * p.geom[24 * p.ne + m];
  for (int d = 0; d < p.nt; ++d) {
    double V, K[3];
#define HB_CALL(N_) near_sep_block<N_>(p, l, m, d, tscale, taylor, etab, V, K)
    HB_NEAR_DISPATCH(HB_CALL)
#undef HB_CALL
    const size_t o = (size_t)d * nnz + ent;
    Vn[o] = V * scale;
    Kn[3 * o] = K[0] * scale;
    Kn[3 * o + 1] = K[1] * scale;
    Kn[3 * o + 2] = K[2] * scale;
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// one wave per touching near pair: tch[e] = (index into the touching list, entry index, local
// vertex of the trial panel for rule vertex 0, 1, 2)
__global__ __launch_bounds__(64) void k_near_touching(const AsmParams *__restrict__ pp,
                                                      const TouchPair *__restrict__ pairs,
                                                      RuleTabs rules,
                                                      const double *__restrict__ tscale,
                                                      const double *__restrict__ taylor,
                                                      const int32_t *__restrict__ tlen,
                                                      const int32_t *__restrict__ tch,
                                                      int64_t nnz, double *__restrict__ Vn,
                                                      double *__restrict__ Kn) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  stage_exp_tab_pos(etab);
  __syncthreads();
  const int32_t *t = tch + 5 * blockIdx.x;
  const TouchPair &tp = pairs[t[0]];
  const int ent = t[1];
  const int cls = __builtin_amdgcn_readfirstlane(tp.cls);
  const double *__restrict__ tab = rules.d[cls];
  const int ntab = rules.n[cls], lane = threadIdx.x;
  for (int d = 0; d < p.nt;) {
    if (d >= p.dsw && d + 1 < p.nt) {
      // Taylor blocks d, d + 1 (d - dsw even: one pass, one polynomial length)
      double V[2], K[2][3];
#define HB_CALL(N_) near_touch_block2<N_>(p, tp, tab, ntab, cls, lane, d, tscale, taylor, etab, V, K)
      HB_NEAR_DISPATCH(HB_CALL)
#undef HB_CALL
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        V[b] = wsum(V[b]);
        K[b][0] = wsum(K[b][0]);
        K[b][1] = wsum(K[b][1]);
        K[b][2] = wsum(K[b][2]);
      }
      if (lane == 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const size_t o = (size_t)(d + b) * nnz + ent;
          Vn[o] = V[b] * tp.scale;
#pragma unroll
          for (int j = 0; j < 3; ++j) Kn[3 * o + t[2 + j]] = K[b][j] * tp.scale;
        }
      }
      d += 2;
      continue;
    }
    double V, K[3];
#define HB_CALL(N_) near_touch_block<N_>(p, tp, tab, ntab, cls, lane, d, tscale, taylor, etab, V, K)
    HB_NEAR_DISPATCH(HB_CALL)
#undef HB_CALL
    V = wsum(V);
    K[0] = wsum(K[0]);
    K[1] = wsum(K[1]);
    K[2] = wsum(K[2]);
    if (lane == 0) {
      const size_t o = (size_t)d * nnz + ent;
      Vn[o] = V * tp.scale;
#pragma unroll
      for (int j = 0; j < 3; ++j) Kn[3 * o + t[2 + j]] = K[j] * tp.scale;
    }
    ++d;
  }
}

}  // namespace

int launch_assemble_near(hb_ctx *c, double *V, double *K, hipStream_t s) {
  if (c->near_nsep > 0)
    hipLaunchKernelGGL(k_near_separated, dim3((unsigned)((c->near_nsep + 255) / 256)), dim3(256), 0,
                       s, c->d_params, c->d_tscale, c->d_taylor, c->d_tlen_sep, c->d_near_sep,
                       (int)c->near_nsep, c->near_nnz, V, K);
  if (c->near_ntouch > 0) {
    RuleTabs rt{};
    for (int k = 1; k <= 3; ++k) {
      rt.d[k] = c->ss[k].d;
      rt.n[k] = c->ss[k].n;
    }
    hipLaunchKernelGGL(k_near_touching, dim3((unsigned)c->near_ntouch), dim3(64), 0, s,
                       c->d_params, c->d_touch, rt, c->d_tscale, c->d_taylor, c->d_tlen_touch,
                       c->d_near_touch, c->near_nnz, V, K);
  }
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

}  // namespace hb
