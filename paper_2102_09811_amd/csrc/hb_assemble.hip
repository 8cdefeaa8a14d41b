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
#include <algorithm>

#include "hb_closed.h"
#include "hb_device.h"
#include "hb_internal.h"
#include "hb_sep.h"

namespace hb {
namespace {

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

// Transposed-order double-layer contribution of a separated pair: row m, trial vertex j, kept
// vertex-major in KT so that the lanes (consecutive m) of a wave add to contiguous addresses.
template <typename TS>
__device__ __forceinline__ void add_block_KT(const AsmParams &p, int d, int m, int j, double v) {
  TS *KT = (TS *)p.KT;
  atomicAdd(&KT[((size_t)d * p.nv + j) * p.ne + m], (TS)v);
}

constexpr int kLC = 2;  // closed-form levels per pass over the quadrature points

// ------------------------------------------------------------------------------------------
// Separated pairs.  Both panels use the same 7-point rule, so the ordered pairs (l, m) and (m, l)
// share all 49 point pairs (r changes sign, rho does not): one lane evaluates the unordered pair
// {l, m} once and emits both orders.  V^d[l][m] = V^d[m][l]; the double layer differs only in the
// normal and the p1 basis:  (l, m) uses r . n_m and the basis at the m-nodes,  (m, l) uses
// -r . n_l and the basis at the l-nodes.  Each wave takes one task from a host list: test panel l
// and up to 64 trial panels m0, m0 + 1, ... modulo E_x (a round-robin pairing: every unordered
// pair occurs once and every row fills whole waves but the last); lane i takes m0 + i.
// ------------------------------------------------------------------------------------------
struct SymSums {
  double V[kLC + 2];
  double K1[kLC + 2][3];  // order (l, m): trial m
  double K2[kLC + 2][3];  // order (m, l): trial l
};

__device__ __forceinline__ void shift_sym(SymSums &S) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    S.V[c] = S.V[kLC + c];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      S.K1[c][q] = S.K1[kLC + c][q];
      S.K2[c][q] = S.K2[kLC + c][q];
    }
  }
#pragma unroll
  for (int j = 2; j < kLC + 2; ++j) {
    S.V[j] = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) S.K1[j][q] = S.K2[j][q] = 0.0;
  }
}

// Blocks completed by the pass over levels i0 .. i0+kLC-1, both orders.
template <typename TS, int D>
__device__ __forceinline__ void emit_sym(const AsmParams &p, int i0, int l, int m,
                                         const int vl[3], const int vm[3], double scale,
                                         const SymSums &S, double sV, const double sK1[3],
                                         const double sK2[3]) {
  const int i1 = min(i0 + kLC - 1, D);
#pragma unroll
  for (int j = 0; j < kLC + 1; ++j) {
    const int d = i0 - 1 + j;
    if (d < 0 || d > i1 - 1 || d >= D || d >= p.nt) continue;
    const int c = d - i0 + 2;
    double v, k1[3], k2[3];
    if (d == 0) {
      v = p.kVs * sV + p.kV * (S.V[c] - S.V[c + 1]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        k1[q] = p.kKs * sK1[q] + p.kK * (S.K1[c + 1][q] - S.K1[c][q]);
        k2[q] = p.kKs * sK2[q] + p.kK * (S.K2[c + 1][q] - S.K2[c][q]);
      }
    } else {
      v = p.kV * (2.0 * S.V[c] - S.V[c + 1] - S.V[c - 1]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        k1[q] = -p.kK * (2.0 * S.K1[c][q] - S.K1[c + 1][q] - S.K1[c - 1][q]);
        k2[q] = -p.kK * (2.0 * S.K2[c][q] - S.K2[c + 1][q] - S.K2[c - 1][q]);
      }
    }
    if (p.do_V) {
      store_block<TS>(p, d, l, m, v * scale);
      store_block<TS>(p, d, m, l, v * scale);
    }
    if (p.do_K) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        add_block_K<TS>(p, d, l, vm[q], k1[q] * scale);
        add_block_KT<TS>(p, d, m, vl[q], k2[q] * scale);
      }
    }
  }
}

// Read-only tables of the separated kernel, passed as restrict kernel arguments so that uniform
// reads (test nodes of l, polynomial coefficients) become scalar loads.
struct SepTabs {
  const double *__restrict__ geom;      // SoA [25][ne]
  const double *__restrict__ tscale;    // [nt][3]
  const double *__restrict__ taylor;    // [nt][2][kTaylorN]
  const float *__restrict__ taylor32;   // [nt][2][kTaylorN32]
  const int *__restrict__ tdeg;         // [nt][2]
  const double *etab;                   // LDS: 2^{-j/64} (exp_neg_t) or 2^{j/256} (exp_neg_m)
  const int *__restrict__ tlen;         // [nt]: length of the double pass from block d (k_separated)
};

// Per-lane data of an unordered separated pair.  The wave's test panel l is uniform: its rule
// nodes sit in LDS (xs[a] = x, y, z, w_a), next to the rule's barycentrics (lam[a] = lambda_0..2,
// w_a), so the inner loop over the test nodes reads them with broadcast LDS loads.
struct SepLane {
  const double *xs;        // LDS [kFarN][4]: test nodes of l and the rule weight
  const double *lam;       // LDS [kFarN][4]: barycentrics of the rule nodes and the weight
  double nm[3], nl[3];     // unit normals of m and l
  double shift;            // inactive lanes integrate a far-away copy and store nothing
};

template <typename TS, int D, int I0>
__device__ __forceinline__ void sym_pass(const AsmParams &p, const SepTabs &T, int l, int m,
                                         const int vl[3], const int vm[3], bool active,
                                         double scale, const SepLane &L, SymSums &S, double &sV,
                                         double sK1[3], double sK2[3]) {
  if constexpr (I0 <= D) {
    const int ne = p.ne;
#pragma unroll 1
    for (int b = 0; b < kFarN; ++b) {
      const double y0 = T.geom[(b * 3 + 0) * ne + m] + L.shift;
      const double y1 = T.geom[(b * 3 + 1) * ne + m];
      const double y2 = T.geom[(b * 3 + 2) * ne + m];
      const RuleNode Lb = rule_node(L.lam, b);
      const double wb = Lb.w;
      double tK[kLC], tsK = 0.0;
#pragma unroll
      for (int j = 0; j < kLC; ++j) tK[j] = 0.0;
#pragma unroll 1
      for (int a = 0; a < kFarN; ++a) {
        const RuleNode X = rule_node(L.xs, a);
        const double rx = X.x - y0;
        const double ry = X.y - y1;
        const double rz = X.z - y2;
        const double rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
        const double rho = sqrt(rho2);
        const double inv_rho = 1.0 / rho;
        const double wa = X.w;
        const double W = wa * wb;
        const double wrn1 = wa * fma(rx, L.nm[0], fma(ry, L.nm[1], rz * L.nm[2]));
        const double wrn2 = -W * fma(rx, L.nl[0], fma(ry, L.nl[1], rz * L.nl[2]));
        const RuleNode La = rule_node(L.lam, a);
        const double la0 = La.x, la1 = La.y, la2 = La.z;
        if constexpr (I0 == 0) {
          sV = fma(W, inv_rho, sV);
          const double i3 = inv_rho * inv_rho * inv_rho;
          tsK = fma(wrn1, i3, tsK);
          const double u = wrn2 * i3;
          sK2[0] = fma(u, la0, sK2[0]);
          sK2[1] = fma(u, la1, sK2[1]);
          sK2[2] = fma(u, la2, sK2[2]);
        }
#pragma unroll
        for (int j = 0; j < kLC; ++j) {
          if (I0 + j > D) continue;
          double rA, kB;
          level_terms(p, I0 + j, rho, inv_rho, rA, kB);
          S.V[2 + j] = fma(W, rA, S.V[2 + j]);
          tK[j] = fma(wrn1, kB, tK[j]);
          const double u = wrn2 * kB;
          S.K2[2 + j][0] = fma(u, la0, S.K2[2 + j][0]);
          S.K2[2 + j][1] = fma(u, la1, S.K2[2 + j][1]);
          S.K2[2 + j][2] = fma(u, la2, S.K2[2 + j][2]);
        }
      }
      const double lb[3] = {Lb.x, Lb.y, Lb.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double phi = wb * lb[k];
#pragma unroll
        for (int j = 0; j < kLC; ++j) S.K1[2 + j][k] = fma(phi, tK[j], S.K1[2 + j][k]);
        if constexpr (I0 == 0) sK1[k] = fma(phi, tsK, sK1[k]);
      }
    }
    if (active) emit_sym<TS, D>(p, I0, l, m, vl, vm, scale, S, sV, sK1, sK2);
    shift_sym(S);
    sym_pass<TS, D, I0 + kLC>(p, T, l, m, vl, vm, active, scale, L, S, sV, sK1, sK2);
  }
}

// Taylor blocks d0 and d0 + 1 of an unordered separated pair (both of polynomial length N; the
// second is a copy of the first when d0 + 1 = nt, and then not stored).  r, rho^2 and the two
// normal products are formed once per point pair for both blocks.  Sums per block: TV (V),
// TK1 (trial m) and TK2 (trial l).  The double layer's polynomial is P - P' of the single
// layer's (K^d / (r . n) = -(alpha / rho) dV^d / drho, term by term in the series), so one
// Horner sweep per block gives both and only the single layer's coefficients are read.
struct TaylorSums {
  double V[2], K1[2][3], K2[2][3];
};

template <int N, bool WCLAMP = false>
__device__ __forceinline__ void sym_taylor2(const AsmParams &p, const SepTabs &T, int d0, int d1,
                                            int m, const SepLane &L, TaylorSums &R) {
  const int ne = p.ne;
  const double c0 = T.tscale[3 * d0 + 2], c1 = T.tscale[3 * d1 + 2];
  const double *cv0 = T.taylor + (size_t)(2 * d0) * kTaylorN;
  const double *cv1 = T.taylor + (size_t)(2 * d1) * kTaylorN;
  // rho^2 clamped where e^{-w} of both blocks is 0 in double anyway (w >= 1000 for the smaller of
  // c0, c1): on uniform grids the other block's w stays below 1000 (d0 + 1) / d0 <= 1334 and both
  // exponentials take their argument unclamped; on non-uniform grids (WCLAMP) the ratio of the
  // two factors is not bounded and the exponentials clamp w themselves
  const double r2max = 1000.0 / fmin(c0, c1);
  // the transposed order's double layer per test node a, weighted by the basis at a after the pass
  double t2[2][kFarN];
#pragma unroll
  for (int a = 0; a < kFarN; ++a) t2[0][a] = t2[1][a] = 0.0;
#pragma unroll 1
  for (int b = 0; b < kFarN; ++b) {
    const double y0 = T.geom[(b * 3 + 0) * ne + m] + L.shift;
    const double y1 = T.geom[(b * 3 + 1) * ne + m];
    const double y2 = T.geom[(b * 3 + 2) * ne + m];
    const RuleNode Lb = rule_node(L.lam, b);
    const double wb = Lb.w;
    double tv0 = 0.0, tv1 = 0.0, tk0 = 0.0, tk1 = 0.0;
#pragma unroll
    for (int a = 0; a < kFarN; ++a) {
      const RuleNode X = rule_node(L.xs, a);
      const double rx = X.x - y0;
      const double ry = X.y - y1;
      const double rz = X.z - y2;
      const double rho2 = fmin(fma(rx, rx, fma(ry, ry, rz * rz)), r2max);
      const double rn1 = fma(rx, L.nm[0], fma(ry, L.nm[1], rz * L.nm[2]));
      const double rn2 = -wb * fma(rx, L.nl[0], fma(ry, L.nl[1], rz * L.nl[2]));
      const double w0 = rho2 * c0, w1 = rho2 * c1;
      // e^{-w} times the test node's weight
      const double e0 = X.w * (WCLAMP ? exp_neg_m(w0, T.etab) : exp_neg_mu(w0, T.etab));
      const double e1 = X.w * (WCLAMP ? exp_neg_m(w1, T.etab) : exp_neg_mu(w1, T.etab));
      double p0, dp0, p1, dp1;
      horner_d<N>(cv0, w0, p0, dp0);
      horner_d<N>(cv1, w1, p1, dp1);
      const double pk0 = (p0 - dp0) * e0, pk1 = (p1 - dp1) * e1;
      tv0 = fma(e0, p0, tv0);
      tv1 = fma(e1, p1, tv1);
      tk0 = fma(rn1, pk0, tk0);
      tk1 = fma(rn1, pk1, tk1);
      t2[0][a] = fma(rn2, pk0, t2[0][a]);
      t2[1][a] = fma(rn2, pk1, t2[1][a]);
    }
    R.V[0] = fma(wb, tv0, R.V[0]);
    R.V[1] = fma(wb, tv1, R.V[1]);
    const double lb[3] = {Lb.x, Lb.y, Lb.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double phi = wb * lb[k];
      R.K1[0][k] = fma(phi, tk0, R.K1[0][k]);
      R.K1[1][k] = fma(phi, tk1, R.K1[1][k]);
    }
  }
#pragma unroll
  for (int a = 0; a < kFarN; ++a) {
    const RuleNode La = rule_node(L.lam, a);
    const double la[3] = {La.x, La.y, La.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R.K2[0][k] = fma(t2[0][a], la[k], R.K2[0][k]);
      R.K2[1][k] = fma(t2[1][a], la[k], R.K2[1][k]);
    }
  }
}

// The same in float (hardware exp, shorter series), accumulated in double per trial node.
template <int N>
__device__ __forceinline__ void sym_taylor2_32(const AsmParams &p, const SepTabs &T, int d0,
                                               int d1, int m, const SepLane &L, TaylorSums &R) {
  const int ne = p.ne;
  const double c0 = T.tscale[3 * d0 + 2], c1 = T.tscale[3 * d1 + 2];
  const float *cv0 = T.taylor32 + (size_t)(2 * d0) * kTaylorN32, *ck0 = cv0 + kTaylorN32;
  const float *cv1 = T.taylor32 + (size_t)(2 * d1) * kTaylorN32, *ck1 = cv1 + kTaylorN32;
#pragma unroll 1
  for (int b = 0; b < kFarN; ++b) {
    const double y0 = T.geom[(b * 3 + 0) * ne + m] + L.shift;
    const double y1 = T.geom[(b * 3 + 1) * ne + m];
    const double y2 = T.geom[(b * 3 + 2) * ne + m];
    const RuleNode Lb = rule_node(L.lam, b);
    const double wb = Lb.w;
    float tv0 = 0.0f, tv1 = 0.0f, tk0 = 0.0f, tk1 = 0.0f;
    float t20[3] = {0.0f, 0.0f, 0.0f}, t21[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int a = 0; a < kFarN; ++a) {
      const RuleNode X = rule_node(L.xs, a);
      const double rx = X.x - y0;
      const double ry = X.y - y1;
      const double rz = X.z - y2;
      const double rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
      const float wa = (float)X.w;
      const float rn1 = wa * (float)fma(rx, L.nm[0], fma(ry, L.nm[1], rz * L.nm[2]));
      const float rn2 = -wa * (float)fma(rx, L.nl[0], fma(ry, L.nl[1], rz * L.nl[2]));
      const float w0 = (float)(rho2 * c0), w1 = (float)(rho2 * c1);
      const float e0 = __expf(-w0), e1 = __expf(-w1);
      const float pk0 = hornerf<N>(ck0, w0) * e0, pk1 = hornerf<N>(ck1, w1) * e1;
      tv0 = fmaf(wa * e0, hornerf<N>(cv0, w0), tv0);
      tv1 = fmaf(wa * e1, hornerf<N>(cv1, w1), tv1);
      tk0 = fmaf(rn1, pk0, tk0);
      tk1 = fmaf(rn1, pk1, tk1);
      const float u0 = rn2 * pk0, u1 = rn2 * pk1;
      const RuleNode La = rule_node(L.lam, a);
      const float la[3] = {(float)La.x, (float)La.y, (float)La.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        t20[k] = fmaf(u0, la[k], t20[k]);
        t21[k] = fmaf(u1, la[k], t21[k]);
      }
    }
    R.V[0] = fma(wb, (double)tv0, R.V[0]);
    R.V[1] = fma(wb, (double)tv1, R.V[1]);
    const double lb[3] = {Lb.x, Lb.y, Lb.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double phi = wb * lb[k];
      R.K1[0][k] = fma(phi, (double)tk0, R.K1[0][k]);
      R.K1[1][k] = fma(phi, (double)tk1, R.K1[1][k]);
      R.K2[0][k] = fma(wb, (double)t20[k], R.K2[0][k]);
      R.K2[1][k] = fma(wb, (double)t21[k], R.K2[1][k]);
    }
  }
}


template <typename TS, int D, bool MIXED>
__global__ __launch_bounds__(256, 2) void k_separated(const AsmParams *__restrict__ pp,
                                                      const double *__restrict__ geom,
                                                      const double *__restrict__ tscale,
                                                      const double *__restrict__ taylor,
                                                      const float *__restrict__ taylor32,
                                                      const int *__restrict__ tdeg,
                                                      const int *__restrict__ tlen,
                                                      const int *__restrict__ tasks,
                                                      const int *__restrict__ tvstart,
                                                      const int *__restrict__ tverts,
                                                      const uint8_t *__restrict__ tslots,
                                                      int ntasks) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  __shared__ double lam[kFarN * 4];
  __shared__ double xs[4][kFarN * 4];
  // the test row's double-layer contributions of the current pass (two blocks) per distinct
  // trial vertex of the wave's task: added in LDS, then once per vertex to K
  __shared__ double kacc[4][2][kSepSlots];
  stage_exp_tab_pos(etab);
  const SepTabs T{geom, tscale, taylor, taylor32, tdeg, etab, tlen};
  // one task per wave: test panel l and up to 64 trial panels m0, m0 + 1, ... (mod E_x); every
  // unordered pair of panels occurs in exactly one task.  Consecutive rows l, l + 1 mirror their V
  // entries into neighbouring columns, so the blocks of one XCD take consecutive tasks.
  const int task = xcd_block() * 4 + (threadIdx.x >> 6);
  const bool valid = task < ntasks;
  const int l = valid ? __builtin_amdgcn_readfirstlane(tasks[3 * task]) : 0;
  stage_test_nodes(p, geom, l, valid, xs[threadIdx.x >> 6], lam);
  __syncthreads();
  if (!valid) return;
  const int lane = threadIdx.x & 63;
  // lanes past the task's count integrate a copy of its first pair and store nothing (they stay
  // for the per-vertex flush of the double layer)
  const bool inrange = lane < __builtin_amdgcn_readfirstlane(tasks[3 * task + 2]);
  const int ne = p.ne;
  int m = __builtin_amdgcn_readfirstlane(tasks[3 * task + 1]) + (inrange ? lane : 0);
  if (m >= ne) m -= ne;
  const int vl[3] = {p.tris[3 * l], p.tris[3 * l + 1], p.tris[3 * l + 2]};
  const int vm[3] = {p.tris[3 * m], p.tris[3 * m + 1], p.tris[3 * m + 2]};
  bool touch = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) touch |= vl[i] == vm[j];
  const bool active = inrange && !touch;
  double(*kw)[kSepSlots] = kacc[threadIdx.x >> 6];
  const int sv0 = __builtin_amdgcn_readfirstlane(tvstart[task]);
  const int nslots = __builtin_amdgcn_readfirstlane(tvstart[task + 1]) - sv0;
  int slot[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) slot[k] = tslots[((size_t)task * 3 + k) * 64 + lane];
  for (int e = lane; e < 2 * kSepSlots; e += 64) kw[e / kSepSlots][e % kSepSlots] = 0.0;
  wave_lds_sync();
  SepLane L;
  L.xs = xs[threadIdx.x >> 6];
  L.lam = lam;
  L.nm[0] = geom[21 * ne + m];
  L.nm[1] = geom[22 * ne + m];
  L.nm[2] = geom[23 * ne + m];
  L.nl[0] = geom[21 * ne + l];
  L.nl[1] = geom[22 * ne + l];
  L.nl[2] = geom[23 * ne + l];
  L.shift = active ? 0.0 : 1.0e3;
  const double scale = geom[24 * ne + l] * geom[24 * ne + m];

  // ---- closed-form levels 0 .. D, kLC per pass ----
  {
    SymSums S;
#pragma unroll
    for (int j = 0; j < kLC + 2; ++j) {
      S.V[j] = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) S.K1[j][q] = S.K2[j][q] = 0.0;
    }
    double sV = 0.0, sK1[3] = {0.0, 0.0, 0.0}, sK2[3] = {0.0, 0.0, 0.0};
    sym_pass<TS, D, 0>(p, T, l, m, vl, vm, active, scale, L, S, sV, sK1, sK2);
  }

  // ---- Taylor blocks d = D .. nt-1, two per pass, with the polynomial length of the pair's
  // first block (the tables hold both blocks at that degree) ----
  for (int d = D; d < p.nt; d += 2) {
    TaylorSums R;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      R.V[j] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) R.K1[j][k] = R.K2[j][k] = 0.0;
    }
    const int d1 = min(d + 1, p.nt - 1);
    if (MIXED && d >= p.mixed_d_min) {
      switch (T.tdeg[2 * d + 1]) {
        case 16: sym_taylor2_32<17>(p, T, d, d1, m, L, R); break;
        case 12: sym_taylor2_32<13>(p, T, d, d1, m, L, R); break;
        case 10: sym_taylor2_32<11>(p, T, d, d1, m, L, R); break;
        case 8: sym_taylor2_32<9>(p, T, d, d1, m, L, R); break;
        case 6: sym_taylor2_32<7>(p, T, d, d1, m, L, R); break;
        default: sym_taylor2_32<5>(p, T, d, d1, m, L, R); break;
      }
    } else {
      // the pass's polynomial length (one of kPolyLens, chosen on the host for this mesh)
      switch (T.tlen[d]) {
        case 5: sym_taylor2<5>(p, T, d, d1, m, L, R); break;
        case 6: sym_taylor2<6>(p, T, d, d1, m, L, R); break;
        case 7: sym_taylor2<7>(p, T, d, d1, m, L, R); break;
        case 8: sym_taylor2<8>(p, T, d, d1, m, L, R); break;
        case 9: sym_taylor2<9>(p, T, d, d1, m, L, R); break;
        case 10: sym_taylor2<10>(p, T, d, d1, m, L, R); break;
        case 11: sym_taylor2<11>(p, T, d, d1, m, L, R); break;
        case 13: sym_taylor2<13>(p, T, d, d1, m, L, R); break;
        case 15: sym_taylor2<15>(p, T, d, d1, m, L, R); break;
        case 17: sym_taylor2<17>(p, T, d, d1, m, L, R); break;
        case 19: sym_taylor2<19>(p, T, d, d1, m, L, R); break;
        case 21: sym_taylor2<21>(p, T, d, d1, m, L, R); break;
        case 25: sym_taylor2<25>(p, T, d, d1, m, L, R); break;
        default: sym_taylor2<29>(p, T, d, d1, m, L, R); break;
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int dj = d + j;
        if (dj >= p.nt) break;
        if (p.do_V) {
          const double v = R.V[j] * T.tscale[3 * dj] * scale;
          store_block<TS>(p, dj, l, m, v);
          store_block<TS>(p, dj, m, l, v);
        }
        if (p.do_K) {
          const double ks = T.tscale[3 * dj + 1] * scale;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            atomicAdd(&kw[j][slot[k]], R.K1[j][k] * ks);
            add_block_KT<TS>(p, dj, m, vl[k], R.K2[j][k] * ks);
          }
        }
      }
    }
    if (p.do_K) {
      // the row's per-vertex sums of this pass to K, each vertex once, and the slots cleared
      wave_lds_sync();
      for (int sidx = lane; sidx < nslots; sidx += 64) {
        const int v = tverts[sv0 + sidx];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double acc = kw[j][sidx];
          if (acc != 0.0 && d + j < p.nt) add_block_K<TS>(p, d + j, l, v, acc);
          kw[j][sidx] = 0.0;
        }
      }
      wave_lds_sync();
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

// Taylor blocks d0 and d0 + 1 of one touching pair (polynomial length N, the second block a copy
// of the first when d0 + 1 = nt): lane partial sums over its rule points, the rule point shared
// by both blocks.
template <int N>
__device__ __forceinline__ void touch_taylor2(const AsmParams &p, const SepTabs &T,
                                              const TouchPair &tp, const double *__restrict__ tab,
                                              int ntab, int lane, int d0, int d1, TaylorSums &R) {
  const double c0 = T.tscale[3 * d0 + 2], c1 = T.tscale[3 * d1 + 2];
  const double *cv0 = T.taylor + (size_t)(2 * d0) * kTaylorN, *ck0 = cv0 + kTaylorN;
  const double *cv1 = T.taylor + (size_t)(2 * d1) * kTaylorN, *ck1 = cv1 + kTaylorN;
#pragma unroll 1
  for (int q = lane; q < ntab; q += 64) {
    const TouchPoint t = touch_point(tp, tab, ntab, q, false);
    const double w0 = t.rho2 * c0, w1 = t.rho2 * c1;
    const double e0 = exp_neg_t(w0, T.etab), e1 = exp_neg_t(w1, T.etab);
    R.V[0] = fma(t.W * e0, horner<N>(cv0, w0), R.V[0]);
    R.V[1] = fma(t.W * e1, horner<N>(cv1, w1), R.V[1]);
    const double u0 = t.wrn * e0 * horner<N>(ck0, w0);
    const double u1 = t.wrn * e1 * horner<N>(ck1, w1);
    R.K1[0][0] = fma(u0, t.l0, R.K1[0][0]);
    R.K1[0][1] = fma(u0, t.l1, R.K1[0][1]);
    R.K1[0][2] = fma(u0, t.l2, R.K1[0][2]);
    R.K1[1][0] = fma(u1, t.l0, R.K1[1][0]);
    R.K1[1][1] = fma(u1, t.l1, R.K1[1][1]);
    R.K1[1][2] = fma(u1, t.l2, R.K1[1][2]);
  }
}

// ------------------------------------------------------------------------------------------
// Touching pairs, one wave per pair: the lanes stride over the regularised rule's points and the
// pair's sums are reduced over the wave, the sixteen sums of a Taylor pass through LDS (each lane
// writes its partial sums, four lanes add up a sum's sixteen-lane quarters and combine them), so
// that the stores are spread over the lanes.  Pairs sharing one vertex are integrated once for
// both orders: the two sub-maps of the vertex rule are each other's x <-> y swap, and the local
// vertex orders depend only on the shared vertex, so the order (m, l) sees the same point pairs
// with r -> -r, trial normal n_l and the trial basis at the x points (V^d[m][l] = V^d[l][m]).
// A list entry is a pair index, ~index for such a pair (SYM launch).
// ------------------------------------------------------------------------------------------
constexpr int kRedRow = 66;  // LDS row of one sum's 64 partial sums (padded against bank conflicts)


// Sum over the wave, left in every lane (bitwise equal): the rows of sixteen lanes as below, then
// the four row sums pairwise.
__device__ __forceinline__ double group_sum(double v);
__device__ __forceinline__ double wave_sum64(double v) {
  v = group_sum(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Sum over the sixteen lanes of a row, left in every lane of the row (bitwise equal): pairs
// (lane ^ 1), quads (lane ^ 2), half rows (mirror within eight lanes), rows (mirror within
// sixteen); each step adds two equal partial sums in either order.
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

// One rule point of a touching pair: r from the edge-vector form, the trial normal product and
// p1 basis, and with SYM those of the order (m, l) as well.  SYM entries are vertex pairs, whose
// rule stores the reference coordinates themselves, c = (x1, x2, -y1, -y2): both barycentric
// triples follow from them, (1 - y1, y1 - y2, y2) and (1 - x1, x1 - x2, x2), instead of being
// loaded (5 table reads per point instead of 11).
template <bool SYM>
struct TouchPt {
  double rho2, W, wrn1, wrn2, l[3], lx[3];
};

template <bool SYM>
__device__ __forceinline__ TouchPt<SYM> touch_pt(const TouchPair &tp, const double nl[3],
                                                 const RuleCols &col, int cls, unsigned q) {
  const unsigned off = 8u * q;
  // the third coordinate is zero in the identical and edge rules (the other entries), the
  // fourth in the identical rule; the edge rule's fourth is -y2, minus the last trial barycentric
  const double a1 = col.at(0, off), a2 = col.at(1, off), a3 = SYM ? col.at(2, off) : 0.0,
               a4 = (!SYM && cls == 3) ? 0.0 : col.at(3, off);
  double rx = a1 * tp.E1[0] + a2 * tp.E2[0], ry = a1 * tp.E1[1] + a2 * tp.E2[1],
         rz = a1 * tp.E1[2] + a2 * tp.E2[2];
  if constexpr (SYM) {
    rx += a3 * tp.F1[0];
    ry += a3 * tp.F1[1];
    rz += a3 * tp.F1[2];
  }
  rx += a4 * tp.F2[0];
  ry += a4 * tp.F2[1];
  rz += a4 * tp.F2[2];
  TouchPt<SYM> t;
  t.rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
  t.W = col.at(4, off);
  t.wrn1 = t.W * fma(rx, tp.n[0], fma(ry, tp.n[1], rz * tp.n[2]));
  if constexpr (SYM) {
    t.l[0] = 1.0 + a3;
    t.l[1] = a4 - a3;
    t.l[2] = -a4;
    t.wrn2 = -t.W * fma(rx, nl[0], fma(ry, nl[1], rz * nl[2]));
    t.lx[0] = 1.0 - a1;
    t.lx[1] = a1 - a2;
    t.lx[2] = a2;
  } else {
    t.l[0] = col.at(5, off);
    t.l[1] = col.at(6, off);
    t.l[2] = cls == 2 ? -a4 : col.at(7, off);
    t.wrn2 = 0.0;
    t.lx[0] = t.lx[1] = t.lx[2] = 0.0;
  }
  return t;
}

// Per-pair data of a wave (uniform); gl: the lane.
struct TouchGroup {
  const TouchPair *tp;
  RuleCols col;
  int cls, ntab, gl, l, m;
  int vtx[3], vtxl[3];
  double nl[3], scale;
};

// Closed-form levels I0 .. I0+kLC-1 of a touching pair (both orders with SYM), then the blocks
// they complete (stored by the group's first lane).
struct TouchLevels {
  double V[kLC + 2], K1[kLC + 2][3], K2[kLC + 2][3];
};

template <typename TS, int D, bool SYM, int I0>
__device__ __forceinline__ void touch_closed(const AsmParams &p, const TouchGroup &G,
                                             TouchLevels &S, double &sV, double sK1[3],
                                             double sK2[3]) {
  if constexpr (I0 <= D) {
#pragma unroll 1
    for (int q = threadIdx.x; q < G.ntab; q += 64) {
      const TouchPt<SYM> t = touch_pt<SYM>(*G.tp, G.nl, G.col, G.cls, q);
      const double rho = sqrt(t.rho2), inv_rho = 1.0 / rho;
      if constexpr (I0 == 0) {
        sV = fma(t.W, inv_rho, sV);
        const double i3 = inv_rho * inv_rho * inv_rho;
        const double u1 = t.wrn1 * i3, u2 = t.wrn2 * i3;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          sK1[k] = fma(u1, t.l[k], sK1[k]);
          if constexpr (SYM) sK2[k] = fma(u2, t.lx[k], sK2[k]);
        }
      }
#pragma unroll
      for (int j = 0; j < kLC; ++j) {
        if (I0 + j > D) continue;
        double rA, kB;
        level_terms(p, I0 + j, rho, inv_rho, rA, kB);
        S.V[2 + j] = fma(t.W, rA, S.V[2 + j]);
        const double u1 = t.wrn1 * kB, u2 = t.wrn2 * kB;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          S.K1[2 + j][k] = fma(u1, t.l[k], S.K1[2 + j][k]);
          if constexpr (SYM) S.K2[2 + j][k] = fma(u2, t.lx[k], S.K2[2 + j][k]);
        }
      }
    }
#pragma unroll
    for (int j = 2; j < kLC + 2; ++j) {
      S.V[j] = wave_sum64(S.V[j]);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        S.K1[j][k] = wave_sum64(S.K1[j][k]);
        if constexpr (SYM) S.K2[j][k] = wave_sum64(S.K2[j][k]);
      }
    }
    if constexpr (I0 == 0) {
      sV = wave_sum64(sV);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sK1[k] = wave_sum64(sK1[k]);
        if constexpr (SYM) sK2[k] = wave_sum64(sK2[k]);
      }
    }
    if (threadIdx.x == 0) {
      const int i1 = min(I0 + kLC - 1, D);
#pragma unroll
      for (int j = 0; j < kLC + 1; ++j) {
        const int d = I0 - 1 + j;  // blocks I0-1 .. i1-1
        if (d < 0 || d > i1 - 1 || d >= D || d >= p.nt) continue;
        const int c = d - I0 + 2;
        double v, k1[3], k2[3];
        if (d == 0) {
          v = p.kVs * sV + p.kV * (S.V[c] - S.V[c + 1]);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            k1[k] = p.kKs * sK1[k] + p.kK * (S.K1[c + 1][k] - S.K1[c][k]);
            k2[k] = p.kKs * sK2[k] + p.kK * (S.K2[c + 1][k] - S.K2[c][k]);
          }
        } else {
          v = p.kV * (2.0 * S.V[c] - S.V[c + 1] - S.V[c - 1]);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            k1[k] = -p.kK * (2.0 * S.K1[c][k] - S.K1[c + 1][k] - S.K1[c - 1][k]);
            k2[k] = -p.kK * (2.0 * S.K2[c][k] - S.K2[c + 1][k] - S.K2[c - 1][k]);
          }
        }
        if (p.do_V) {
          store_block<TS>(p, d, G.l, G.m, v * G.scale);
          if constexpr (SYM) store_block<TS>(p, d, G.m, G.l, v * G.scale);
        }
        if (p.do_K) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            add_block_K<TS>(p, d, G.l, G.vtx[k], k1[k] * G.scale);
            if constexpr (SYM) add_block_K<TS>(p, d, G.m, G.vtxl[k], k2[k] * G.scale);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      S.V[c] = S.V[kLC + c];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        S.K1[c][k] = S.K1[kLC + c][k];
        S.K2[c][k] = S.K2[kLC + c][k];
      }
    }
#pragma unroll
    for (int j = 2; j < kLC + 2; ++j) {
      S.V[j] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) S.K1[j][k] = S.K2[j][k] = 0.0;
    }
    touch_closed<TS, D, SYM, I0 + kLC>(p, G, S, sV, sK1, sK2);
  }
}

// Taylor blocks d0 and d1 (= d0 + 1, or d0 at the end) of a touching pair: this lane's partial
// sums over its rule points (single-layer polynomial P, double layer P - P').  R[0], R[1]: V of
// the two blocks; R[2..7]: double-layer parts (block, trial vertex); with SYM R[10..15]: those
// of the order (m, l).
template <bool SYM, int N>
__device__ __forceinline__ void touch_taylor(const SepTabs &T, const TouchGroup &G, int d0, int d1,
                                             double R[16]) {
  const double c0 = T.tscale[3 * d0 + 2], c1 = T.tscale[3 * d1 + 2];
  const double *cv0 = T.taylor + (size_t)(2 * d0) * kTaylorN;
  const double *cv1 = T.taylor + (size_t)(2 * d1) * kTaylorN;
#pragma unroll 1
  for (int q = G.gl; q < G.ntab; q += 64) {
    const TouchPt<SYM> t = touch_pt<SYM>(*G.tp, G.nl, G.col, G.cls, q);
    const double w0 = t.rho2 * c0, w1 = t.rho2 * c1;
    const double e0 = exp_neg_m(w0, T.etab), e1 = exp_neg_m(w1, T.etab);
    double p0, dp0, p1, dp1;
    horner_d<N>(cv0, w0, p0, dp0);
    horner_d<N>(cv1, w1, p1, dp1);
    const double k0 = (p0 - dp0) * e0, k1 = (p1 - dp1) * e1;
    R[0] = fma(t.W * e0, p0, R[0]);
    R[1] = fma(t.W * e1, p1, R[1]);
    const double u10 = t.wrn1 * k0, u11 = t.wrn1 * k1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R[2 + k] = fma(u10, t.l[k], R[2 + k]);
      R[5 + k] = fma(u11, t.l[k], R[5 + k]);
    }
    if constexpr (SYM) {
      const double u20 = t.wrn2 * k0, u21 = t.wrn2 * k1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        R[10 + k] = fma(u20, t.lx[k], R[10 + k]);
        R[13 + k] = fma(u21, t.lx[k], R[13 + k]);
      }
    }
  }
}

// One list entry (a wave): ent indexes pairs (SYM: ~index of a vertex pair, both orders).
template <typename TS, int D, bool SYM>
__device__ __forceinline__ void touch_entry(const AsmParams &p, const TouchPair *__restrict__ pairs,
                                            int ent, const RuleTabs &rules,
                                            const double *__restrict__ tscale,
                                            const double *__restrict__ taylor,
                                            const int *__restrict__ tlen, const double *etab,
                                            double *red) {
  const SepTabs T{nullptr, tscale, taylor, nullptr, nullptr, etab};
  TouchGroup G;
  const TouchPair &tp = pairs[SYM ? ~ent : ent];
  G.tp = &tp;
  const int cls = __builtin_amdgcn_readfirstlane(tp.cls);
  G.cls = cls;
  G.ntab = rules.n[cls];
  G.col = RuleCols(rules.d[cls], G.ntab);
  G.gl = threadIdx.x;
  G.l = tp.l;
  G.m = tp.m;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G.vtx[k] = tp.vtx[k];
    G.vtxl[k] = tp.vtxl[k];
    G.nl[k] = SYM ? p.geom[(21 + k) * p.ne + G.l] : 0.0;
  }
  G.scale = tp.scale;

  {
    TouchLevels S;
#pragma unroll
    for (int j = 0; j < kLC + 2; ++j) {
      S.V[j] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) S.K1[j][k] = S.K2[j][k] = 0.0;
    }
    double sV = 0.0, sK1[3] = {0.0, 0.0, 0.0}, sK2[3] = {0.0, 0.0, 0.0};
    touch_closed<TS, D, SYM, 0>(p, G, S, sV, sK1, sK2);
  }

  // Taylor blocks two per pass.  Sum i of the pass ends in lane 4 i, which stores it: 0, 1 V^d[l][m]
  // of the two blocks, 2..7 their double-layer parts (block, trial vertex), and with SYM 8, 9
  // V^d[m][l] (the sums 0, 1 again) and 10..15 the parts of the order (m, l).
  const int lane = threadIdx.x;
  const int i4 = lane >> 2;
  const int j = i4 < 8 ? (i4 < 2 ? i4 : (i4 - 2) / 3) : (i4 < 10 ? i4 - 8 : (i4 - 10) / 3);
  const int kk = i4 < 2 ? 0 : (i4 < 8 ? (i4 - 2) % 3 : (i4 < 10 ? 0 : (i4 - 10) % 3));
  const bool isV = i4 < 2 || (i4 >= 8 && i4 < 10);
  const int row = i4 < 8 ? G.l : G.m;
  const int col = isV ? (i4 < 8 ? G.m : G.l) : (i4 < 8 ? G.vtx[kk] : G.vtxl[kk]);
  const bool mine = (lane & 3) == 0 && (i4 < 8 || SYM) && (isV ? p.do_V : p.do_K);
  const int src = (i4 == 8 || i4 == 9) ? i4 - 8 : i4;
  for (int d = D; d < p.nt; d += 2) {
    const int d1 = min(d + 1, p.nt - 1);
    double R[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) R[i] = 0.0;
    // the pass's polynomial length (one of kPolyLens, chosen on the host for this mesh)
    switch (tlen[d]) {
      case 5: touch_taylor<SYM, 5>(T, G, d, d1, R); break;
      case 6: touch_taylor<SYM, 6>(T, G, d, d1, R); break;
      case 7: touch_taylor<SYM, 7>(T, G, d, d1, R); break;
      case 8: touch_taylor<SYM, 8>(T, G, d, d1, R); break;
      case 9: touch_taylor<SYM, 9>(T, G, d, d1, R); break;
      case 10: touch_taylor<SYM, 10>(T, G, d, d1, R); break;
      case 11: touch_taylor<SYM, 11>(T, G, d, d1, R); break;
      case 13: touch_taylor<SYM, 13>(T, G, d, d1, R); break;
      case 15: touch_taylor<SYM, 15>(T, G, d, d1, R); break;
      case 17: touch_taylor<SYM, 17>(T, G, d, d1, R); break;
      case 19: touch_taylor<SYM, 19>(T, G, d, d1, R); break;
      case 21: touch_taylor<SYM, 21>(T, G, d, d1, R); break;
      case 25: touch_taylor<SYM, 25>(T, G, d, d1, R); break;
      default: touch_taylor<SYM, 29>(T, G, d, d1, R); break;
    }
    // partial sums to LDS, row i = sum i (R[8], R[9] are unused), padded rows against conflicts
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i != 8 && i != 9 && (SYM || i < 8)) red[i * kRedRow + lane] = R[i];
    __syncthreads();
    const double *q = red + src * kRedRow + 16 * (lane & 3);
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 16; k += 2) {
      const double2 a = *(const double2 *)(q + k);
      v += a.x + a.y;
    }
    v += dpp_d<0xB1>(v);  // the four quarters: quad_perm [1, 0, 3, 2], then [2, 3, 0, 1]
    v += dpp_d<0x4E>(v);
    __syncthreads();
    const int dj = d + j;
    if (mine && dj < p.nt) {
      if (isV) {
        store_block<TS>(p, dj, row, col, v * T.tscale[3 * dj] * G.scale);
      } else {
        add_block_K<TS>(p, dj, row, col, v * T.tscale[3 * dj + 1] * G.scale);
      }
    }
  }
}

// All touching pairs in one launch, one wave per list entry: the first n0 entries are identical
// and edge-sharing pairs (one order each), the rest vertex-sharing pairs (both orders).  The
// longest entries come first (identical pairs have the largest rule), so the short vertex-pair
// waves fill the machine at the end instead of each class leaving its own partial last round.
template <typename TS, int D>
__global__ __launch_bounds__(64, 3) void k_touching(const AsmParams *__restrict__ pp,
                                                    const TouchPair *__restrict__ pairs,
                                                    const int32_t *__restrict__ list, int n0,
                                                    RuleTabs rules,
                                                    const double *__restrict__ tscale,
                                                    const double *__restrict__ taylor,
                                                    const int *__restrict__ tlen) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  __shared__ __align__(16) double red[16 * kRedRow];
  stage_exp_tab_pos(etab);
  __syncthreads();
  const int ent = __builtin_amdgcn_readfirstlane(list[blockIdx.x]);
  if ((int)blockIdx.x < n0)
    touch_entry<TS, D, false>(p, pairs, ent, rules, tscale, taylor, tlen, etab, red);
  else
    touch_entry<TS, D, true>(p, pairs, ent, rules, tscale, taylor, tlen, etab, red);
}

// ------------------------------------------------------------------------------------------
// Non-uniform time grids: blocks V^{k,i}, K^{k,i} (0 <= i <= k < E_t) at packed index
// k (k + 1) / 2 + i, on the same rules and pair lists as the uniform kernels.  A closed block is,
// per point pair, the signed sum of the brackets at its levels: the four-term difference
// F(t_k - t_i) + F(t_{k+1} - t_{i+1}) - F(t_{k+1} - t_i) - F(t_k - t_{i+1}) of
// F = G^{dtau dt} (Sec. 3.1) and of its normal derivative (Sec. 3.2), and on the diagonal
// F(0) - F(h_k) plus h_k G^{dtau}(rho, 0).  A Taylor block is the even series of the
// trapezoid-weighted kernel about the centre of its support, evaluated like the uniform Taylor
// blocks (sym_taylor2 / touch_taylor2) from a list, two entries per pass.  Double storage only.
// ------------------------------------------------------------------------------------------

// Signed level sums of closed block cb at one point pair: sA = sum sg rho A(z), sB = sum sg B(z)/rho.
__device__ __forceinline__ void nu_closed_point(const AsmParams &p, const NuClosed &cb, double rho,
                                                double inv_rho, double &sA, double &sB) {
  sA = 0.0;
  sB = 0.0;
#pragma unroll
  for (int j = 0; j < kNuLev; ++j) {
    if (j >= cb.nlev) break;
    double rA, kB;
    if (cb.c[j] == 0.0) {  // delta = 0: A = B = 1
      rA = rho;
      kB = inv_rho;
    } else {
      closed_level_at(p, cb.c[j], cb.s2[j], cb.s1[j], cb.t2[j], rho, inv_rho, rA, kB);
    }
    sA = fma(cb.sg[j], rA, sA);
    sB = fma(cb.sg[j], kB, sB);
  }
}

// Taylor entries b and b1 (= b + 1, or b itself at the end of the list) of an unordered
// separated pair, with the polynomial length of entry b.
__device__ __forceinline__ void nu_sym_taylor(const AsmParams &p, const SepTabs &T, int b, int b1,
                                              int m, const SepLane &L, TaylorSums &R) {
  switch (T.tdeg[2 * b]) {  // the pass's length for separated pairs, one of kPolyLens
    case 5: sym_taylor2<5, true>(p, T, b, b1, m, L, R); break;
    case 6: sym_taylor2<6, true>(p, T, b, b1, m, L, R); break;
    case 7: sym_taylor2<7, true>(p, T, b, b1, m, L, R); break;
    case 8: sym_taylor2<8, true>(p, T, b, b1, m, L, R); break;
    case 9: sym_taylor2<9, true>(p, T, b, b1, m, L, R); break;
    case 10: sym_taylor2<10, true>(p, T, b, b1, m, L, R); break;
    case 11: sym_taylor2<11, true>(p, T, b, b1, m, L, R); break;
    case 13: sym_taylor2<13, true>(p, T, b, b1, m, L, R); break;
    case 15: sym_taylor2<15, true>(p, T, b, b1, m, L, R); break;
    case 17: sym_taylor2<17, true>(p, T, b, b1, m, L, R); break;
    case 19: sym_taylor2<19, true>(p, T, b, b1, m, L, R); break;
    case 21: sym_taylor2<21, true>(p, T, b, b1, m, L, R); break;
    case 25: sym_taylor2<25, true>(p, T, b, b1, m, L, R); break;
    default: sym_taylor2<29, true>(p, T, b, b1, m, L, R); break;
  }
}

__global__ __launch_bounds__(256, 2) void k_nu_separated(const AsmParams *__restrict__ pp, NuTabs nu,
                                                         const int *__restrict__ tasks,
                                                         int ntasks) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  __shared__ double lam[kFarN * 4];
  __shared__ double xs[4][kFarN * 4];
  stage_exp_tab_pos(etab);
  const double *__restrict__ geom = p.geom;
  const SepTabs T{geom, nu.tscale, nu.taylor, nullptr, nu.tdeg, etab};
  // task list and lane mapping of k_separated: test panel l, trial panels m0 + lane (mod E_x)
  const int task = xcd_block() * 4 + (threadIdx.x >> 6);
  const bool valid = task < ntasks;
  const int l = valid ? __builtin_amdgcn_readfirstlane(tasks[3 * task]) : 0;
  stage_test_nodes(p, geom, l, valid, xs[threadIdx.x >> 6], lam);
  __syncthreads();
  if (!valid) return;
  const int lane = threadIdx.x & 63;
  if (lane >= __builtin_amdgcn_readfirstlane(tasks[3 * task + 2])) return;
  const int ne = p.ne;
  int m = __builtin_amdgcn_readfirstlane(tasks[3 * task + 1]) + lane;
  if (m >= ne) m -= ne;
  const int vl[3] = {p.tris[3 * l], p.tris[3 * l + 1], p.tris[3 * l + 2]};
  const int vm[3] = {p.tris[3 * m], p.tris[3 * m + 1], p.tris[3 * m + 2]};
  bool touch = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) touch |= vl[i] == vm[j];
  const bool active = !touch;
  SepLane L;
  L.xs = xs[threadIdx.x >> 6];
  L.lam = lam;
  L.nm[0] = geom[21 * ne + m];
  L.nm[1] = geom[22 * ne + m];
  L.nm[2] = geom[23 * ne + m];
  L.nl[0] = geom[21 * ne + l];
  L.nl[1] = geom[22 * ne + l];
  L.nl[2] = geom[23 * ne + l];
  L.shift = active ? 0.0 : 1.0e3;
  const double scale = geom[24 * ne + l] * geom[24 * ne + m];

  // ---- closed blocks, one per pass over the 49 point pairs ----
#pragma unroll 1
  for (int cbi = 0; cbi < nu.n_closed; ++cbi) {
    const NuClosed &cb = nu.closed[cbi];
    const bool diag = cb.diag != 0;
    double sV = 0.0, gV = 0.0, sK1[3] = {0.0, 0.0, 0.0}, sK2[3] = {0.0, 0.0, 0.0};
    double gK1[3] = {0.0, 0.0, 0.0}, gK2[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int b = 0; b < kFarN; ++b) {
      const double y0 = geom[(b * 3 + 0) * ne + m] + L.shift;
      const double y1 = geom[(b * 3 + 1) * ne + m];
      const double y2 = geom[(b * 3 + 2) * ne + m];
      const RuleNode Lb = rule_node(L.lam, b);
      const double wb = Lb.w;
      double tK = 0.0, tg = 0.0;
#pragma unroll 1
      for (int a = 0; a < kFarN; ++a) {
        const RuleNode X = rule_node(L.xs, a);
        const double rx = X.x - y0;
        const double ry = X.y - y1;
        const double rz = X.z - y2;
        const double rho = sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
        const double inv_rho = 1.0 / rho;
        const double wa = X.w;
        const RuleNode La = rule_node(L.lam, a);
        const double la[3] = {La.x, La.y, La.z};
        const double W = wa * wb;
        const double wrn1 = wa * fma(rx, L.nm[0], fma(ry, L.nm[1], rz * L.nm[2]));
        const double wrn2 = -W * fma(rx, L.nl[0], fma(ry, L.nl[1], rz * L.nl[2]));
        double sA, sB;
        nu_closed_point(p, cb, rho, inv_rho, sA, sB);
        sV = fma(W, sA, sV);
        tK = fma(wrn1, sB, tK);
        const double u = wrn2 * sB;
#pragma unroll
        for (int k = 0; k < 3; ++k) sK2[k] = fma(u, la[k], sK2[k]);
        if (diag) {
          gV = fma(W, inv_rho, gV);
          const double i3 = inv_rho * inv_rho * inv_rho;
          tg = fma(wrn1, i3, tg);
          const double u3 = wrn2 * i3;
#pragma unroll
          for (int k = 0; k < 3; ++k) gK2[k] = fma(u3, la[k], gK2[k]);
        }
      }
      const double lb[3] = {Lb.x, Lb.y, Lb.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double phi = wb * lb[k];
        sK1[k] = fma(phi, tK, sK1[k]);
        gK1[k] = fma(phi, tg, gK1[k]);
      }
    }
    if (active) {
      const double dV = diag ? cb.kVs : 0.0, dK = diag ? cb.kKs : 0.0;
      const double v = (dV * gV + p.kV * sV) * scale;
      if (p.do_V) {
        store_block<double>(p, cb.out, l, m, v);
        store_block<double>(p, cb.out, m, l, v);
      }
      if (p.do_K) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          add_block_K<double>(p, cb.out, l, vm[k], (dK * gK1[k] - p.kK * sK1[k]) * scale);
          add_block_KT<double>(p, cb.out, m, vl[k], (dK * gK2[k] - p.kK * sK2[k]) * scale);
        }
      }
    }
  }

  // ---- Taylor blocks, two list entries per pass ----
#pragma unroll 1
  for (int b = 0; b < nu.n_taylor; b += 2) {
    const int b1 = min(b + 1, nu.n_taylor - 1);
    TaylorSums R;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      R.V[j] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) R.K1[j][k] = R.K2[j][k] = 0.0;
    }
    nu_sym_taylor(p, T, b, b1, m, L, R);
    if (active) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int bj = b + j;
        if (bj >= nu.n_taylor) break;
        const int out = nu.tout[bj];
        if (p.do_V) {
          const double v = R.V[j] * T.tscale[3 * bj] * scale;
          store_block<double>(p, out, l, m, v);
          store_block<double>(p, out, m, l, v);
        }
        if (p.do_K) {
          const double ks = T.tscale[3 * bj + 1] * scale;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            add_block_K<double>(p, out, l, vm[k], R.K1[j][k] * ks);
            add_block_KT<double>(p, out, m, vl[k], R.K2[j][k] * ks);
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(64, 3) void k_nu_touching(const AsmParams *__restrict__ pp,
                                                       const TouchPair *__restrict__ pairs,
                                                       RuleTabs rules, NuTabs nu) {
  const AsmParams &p = *pp;
  __shared__ double etab[64];
  stage_exp_tab(etab);
  __syncthreads();
  const SepTabs T{nullptr, nu.tscale, nu.taylor, nullptr, nu.tdeg, etab};
  const TouchPair &tp = pairs[blockIdx.x];
  const int cls = __builtin_amdgcn_readfirstlane(tp.cls);
  const double *__restrict__ tab = rules.d[cls];
  const int ntab = rules.n[cls];
  const int lane = threadIdx.x;
  const int l = tp.l, m = tp.m;
  const int vtx[3] = {tp.vtx[0], tp.vtx[1], tp.vtx[2]};

#pragma unroll 1
  for (int cbi = 0; cbi < nu.n_closed; ++cbi) {
    const NuClosed &cb = nu.closed[cbi];
    const bool diag = cb.diag != 0;
    double sV = 0.0, gV = 0.0, sK[3] = {0.0, 0.0, 0.0}, gK[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int q = lane; q < ntab; q += 64) {
      const TouchPoint t = touch_point(tp, tab, ntab, q, true);
      double sA, sB;
      nu_closed_point(p, cb, t.rho, t.inv_rho, sA, sB);
      sV = fma(t.W, sA, sV);
      const double u = t.wrn * sB;
      sK[0] = fma(u, t.l0, sK[0]);
      sK[1] = fma(u, t.l1, sK[1]);
      sK[2] = fma(u, t.l2, sK[2]);
      if (diag) {
        gV = fma(t.W, t.inv_rho, gV);
        const double u3 = t.wrn * t.inv_rho * t.inv_rho * t.inv_rho;
        gK[0] = fma(u3, t.l0, gK[0]);
        gK[1] = fma(u3, t.l1, gK[1]);
        gK[2] = fma(u3, t.l2, gK[2]);
      }
    }
    sV = wave_sum(sV);
#pragma unroll
    for (int k = 0; k < 3; ++k) sK[k] = wave_sum(sK[k]);
    if (diag) {
      gV = wave_sum(gV);
#pragma unroll
      for (int k = 0; k < 3; ++k) gK[k] = wave_sum(gK[k]);
    }
    if (lane == 0) {
      const double dV = diag ? cb.kVs : 0.0, dK = diag ? cb.kKs : 0.0;
      if (p.do_V) store_block<double>(p, cb.out, l, m, (dV * gV + p.kV * sV) * tp.scale);
      if (p.do_K) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
          add_block_K<double>(p, cb.out, l, vtx[k], (dK * gK[k] - p.kK * sK[k]) * tp.scale);
      }
    }
  }

#pragma unroll 1
  for (int b = 0; b < nu.n_taylor; b += 2) {
    const int b1 = min(b + 1, nu.n_taylor - 1);
    TaylorSums R;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      R.V[j] = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) R.K1[j][k] = 0.0;
    }
    switch (T.tdeg[2 * b + 1]) {  // the pass's length for touching pairs, one of kPolyLens
      case 5: touch_taylor2<5>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 6: touch_taylor2<6>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 7: touch_taylor2<7>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 8: touch_taylor2<8>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 9: touch_taylor2<9>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 10: touch_taylor2<10>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 11: touch_taylor2<11>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 13: touch_taylor2<13>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 15: touch_taylor2<15>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 17: touch_taylor2<17>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 19: touch_taylor2<19>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 21: touch_taylor2<21>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      case 25: touch_taylor2<25>(p, T, tp, tab, ntab, lane, b, b1, R); break;
      default: touch_taylor2<29>(p, T, tp, tab, ntab, lane, b, b1, R); break;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      R.V[j] = wave_sum(R.V[j]);
#pragma unroll
      for (int k = 0; k < 3; ++k) R.K1[j][k] = wave_sum(R.K1[j][k]);
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int bj = b + j;
        if (bj >= nu.n_taylor) break;
        const int out = nu.tout[bj];
        if (p.do_V) store_block<double>(p, out, l, m, R.V[j] * T.tscale[3 * bj] * tp.scale);
        if (p.do_K) {
          const double ks = T.tscale[3 * bj + 1] * tp.scale;
#pragma unroll
          for (int k = 0; k < 3; ++k) add_block_K<double>(p, out, l, vtx[k], R.K1[j][k] * ks);
        }
      }
    }
  }
}

}  // namespace

void launch_nu_separated(const AsmParams *dp, const NuTabs &nu, const int32_t *tasks,
                         int64_t ntasks, hipStream_t s) {
  hipLaunchKernelGGL(k_nu_separated, dim3((unsigned)((ntasks + 3) / 4)), dim3(256), 0, s, dp, nu,
                     tasks, (int)ntasks);
}

void launch_nu_touching(const AsmParams *dp, const NuTabs &nu, const TouchPair *pairs,
                        int64_t npairs, const SSRule rules[4], hipStream_t s) {
  RuleTabs rule{};
  for (int c = 1; c <= 3; ++c) {
    rule.d[c] = rules[c].d;
    rule.n[c] = rules[c].n;
  }
  hipLaunchKernelGGL(k_nu_touching, dim3((unsigned)npairs), dim3(64), 0, s, dp, pairs, rule, nu);
}

struct SepTasks {
  const int32_t *tasks, *vstart, *verts;
  const uint8_t *slots;
  int n;
};

template <typename TS, int D>
static void launch_sep(dim3 grid, hipStream_t s, const AsmParams *dp, const AsmParams &hp,
                       const SepTasks &t, bool mixed) {
  if (mixed)
    hipLaunchKernelGGL((k_separated<TS, D, true>), grid, dim3(256), 0, s, dp, hp.geom, hp.tscale,
                       hp.taylor, hp.taylor32, hp.tdeg, hp.tlen_sep, t.tasks, t.vstart, t.verts, t.slots, t.n);
  else
    hipLaunchKernelGGL((k_separated<TS, D, false>), grid, dim3(256), 0, s, dp, hp.geom, hp.tscale,
                       hp.taylor, hp.taylor32, hp.tdeg, hp.tlen_sep, t.tasks, t.vstart, t.verts, t.slots, t.n);
}

void launch_assemble_separated(const AsmParams *dp, const AsmParams &p, const int32_t *tasks,
                               const int32_t *vstart, const int32_t *verts, const uint8_t *slots,
                               int64_t ntasks, int precision, int storage_f32, hipStream_t s) {
  dim3 grid((unsigned)((ntasks + 3) / 4));
  const SepTasks t{tasks, vstart, verts, slots, (int)ntasks};
  const bool mixed = precision == HB_PREC_MIXED;
  switch (p.dsw) {
    case 16:
      if (storage_f32) launch_sep<float, 16>(grid, s, dp, p, t, mixed);
      else launch_sep<double, 16>(grid, s, dp, p, t, mixed);
      break;
    case 8:
      if (storage_f32) launch_sep<float, 8>(grid, s, dp, p, t, mixed);
      else launch_sep<double, 8>(grid, s, dp, p, t, mixed);
      break;
    default:
      if (storage_f32) launch_sep<float, 3>(grid, s, dp, p, t, mixed);
      else launch_sep<double, 3>(grid, s, dp, p, t, mixed);
      break;
  }
}

// K[d][m][j] += KT[d][j][m] through a 64 x 64 tile in LDS, coalesced on both sides.
template <typename TS>
__global__ __launch_bounds__(256) void k_fold_KT(const TS *__restrict__ KT, TS *__restrict__ K,
                                                 int ne, int nv, int nt) {
  __shared__ TS tile[64][65];
  const int j0 = blockIdx.x * 64, m0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int d = blockIdx.z; d < nt; d += gridDim.z) {
    const TS *src = KT + (size_t)d * nv * ne;
    TS *dst = K + (size_t)d * ne * nv;
    for (int r = ty; r < 64; r += 4) {
      const int j = j0 + r, m = m0 + tx;
      tile[r][tx] = (j < nv && m < ne) ? src[(size_t)j * ne + m] : TS(0);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
      const int m = m0 + r, j = j0 + tx;
      if (m < ne && j < nv) dst[(size_t)m * nv + j] += tile[tx][r];
    }
    __syncthreads();
  }
}

void launch_fold_KT(const AsmParams &p, int storage_f32, hipStream_t s) {
  dim3 grid((p.nv + 63) / 64, (p.ne + 63) / 64, std::min(p.nt, 4096));
  if (storage_f32)
    hipLaunchKernelGGL(k_fold_KT<float>, grid, dim3(256), 0, s, (const float *)p.KT,
                       (float *)p.K, p.ne, p.nv, p.nt);
  else
    hipLaunchKernelGGL(k_fold_KT<double>, grid, dim3(256), 0, s, (const double *)p.KT,
                       (double *)p.K, p.ne, p.nv, p.nt);
}

template <typename TS, int D>
static void launch_touch(hipStream_t s, const AsmParams *dp, const AsmParams &hp,
                         const TouchPair *pairs, const int32_t *list, int nlist, int nsym,
                         const RuleTabs &rule) {
  const int n0 = nlist - nsym;
  if (nlist > 0)
    hipLaunchKernelGGL((k_touching<TS, D>), dim3(nlist), dim3(64), 0, s, dp, pairs, list, n0, rule,
                       hp.tscale, hp.taylor, hp.tlen_touch);
}

void launch_assemble_touching(const AsmParams *dp, const AsmParams &p, const TouchPair *pairs,
                              const int32_t *list, int64_t nlist, int64_t nsym,
                              const SSRule rules[4], int storage_f32, hipStream_t s) {
  const int n = (int)nlist, ns = (int)nsym;
  RuleTabs rule{};
  for (int c = 1; c <= 3; ++c) {
    rule.d[c] = rules[c].d;
    rule.n[c] = rules[c].n;
  }
  switch (p.dsw) {
    case 16:
      if (storage_f32) launch_touch<float, 16>(s, dp, p, pairs, list, n, ns, rule);
      else launch_touch<double, 16>(s, dp, p, pairs, list, n, ns, rule);
      break;
    case 8:
      if (storage_f32) launch_touch<float, 8>(s, dp, p, pairs, list, n, ns, rule);
      else launch_touch<double, 8>(s, dp, p, pairs, list, n, ns, rule);
      break;
    default:
      if (storage_f32) launch_touch<float, 3>(s, dp, p, pairs, list, n, ns, rule);
      else launch_touch<double, 3>(s, dp, p, pairs, list, n, ns, rule);
      break;
  }
}

}  // namespace hb
