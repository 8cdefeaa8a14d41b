// Hypersingular operator of the heat equation (Sec. 3.3): D_h^d = D_h^{1,d} + D_h^{2,d}, and the
// blockwise transpose used for K_h^T in the Neumann system (Sec. 3.4).
//
// D^{2,d}(r), the kernel of the second part (Sec. 3.3, eq. for D^{2,d}), with z_i = rho / (2 sqrt(
// alpha i h)) and int_0^delta G(r, s) ds = erfc(z) / (4 pi alpha rho):
//   d = 0:  alpha int_0^h G = erfc(z_1) / (4 pi rho);
//   d >= 1: alpha [int_{dh}^{(d+1)h} G - int_{(d-1)h}^{dh} G]
//         = [erfc(z_{d+1}) - 2 erfc(z_d) + erfc(z_{d-1})] / (4 pi rho),  erfc(z_0) = 0,
//     taken as minus the same difference of erf when z_{d-1} < 1 (the erfc values then sit near 1);
//   d >= kD2Closed: the same integral as alpha h int_{-1}^{1} sgn(u) G(r, (d+u) h) du, expanded in
//     u around dh.  Only odd derivatives survive: with f(s) = s^{-3/2} e^{-a/s},
//     f^{(n)}(s) = s^{-3/2-n} e^{-w} Q_n(w) (w = rho^2 / (4 alpha d h)), so
//     D^{2,d} = alpha h G(r, dh) sum_k 2 d^{-(2k+1)} Q_{2k+1}(w) / (2k+2)!,
//     a polynomial in w tabulated on the host; no cancelling differences remain.
// Blocks (Sec. 3.3, Galerkin matrix D_h^2): p1 test x p1 trial with n(x) . n(y), the same rules as
// V_h.  Separated pairs: the task list of the V_h / K_h assembly (test panel l and up to 64
// trial panels, each unordered pair once), Radon's rule on both panels, contributions added to
// the workspace row block of l; then D^2 = W + W^T.  Touching pairs: one wave per pair (vertex
// pairs once for both orders), the regularised rule of its class.
// D_h^{1,d} = T^T (alpha^2 V^d (x) I_3) T (Sec. 3.3, eq. for D_h^{1,d}) is added entry by entry
// from V_h^d and the surface curls of the local p1 basis.
// The same p1 x p1 kernels assemble V_h^{11}, the single layer between p1 functions (the matrix
// of the paper's preconditioner for D_h, Sec. 6.1), with the kernel V^d(r) of V_h: closed form
// (second differences of G^{dtau dt} = rho A(z) / (8 pi alpha^2)) below d_switch, the even Taylor
// tables of V_h above, and no normal factor.
#include "hb_closed.h"
#include "hb_device.h"
#include "hb_internal.h"
#include "hb_sep.h"

namespace hb {
namespace {

constexpr double kInv4Pi = 0.079577471545947667884;

// z at level i is rho p.lv.c[i] (c[i] = 1 / (2 sqrt(alpha i h)), tabulated per context)
static_assert(kD2Closed <= kMaxClosed, "the closed-form D^2 blocks read levels up to kD2Closed");
__device__ __forceinline__ double d2_closed(const AsmParams &p, double rho, int d) {
  const double c = kInv4Pi / rho;
  const double zp = rho * p.lv.c[d + 1];
  if (d == 0) return erfc(zp) * c;
  const double z0 = rho * p.lv.c[d];
  if (d == 1) return (erfc(zp) - 2.0 * erfc(z0)) * c;
  const double zm = rho * p.lv.c[d - 1];
  if (zm < 1.0) return -(erf(zp) - 2.0 * erf(z0) + erf(zm)) * c;
  return (erfc(zp) - 2.0 * erfc(z0) + erfc(zm)) * c;
}

constexpr int kKindV11 = 0, kKindD2 = 1;

// rho A(z) at level i (G^{dtau dt}(rho, i h) = kV rho A(z))
__device__ __forceinline__ double rA_level(const AsmParams &p, int i, double rho, double inv_rho) {
  double rA, kB;
  level_terms(p, i, rho, inv_rho, rA, kB);
  return rA;
}

// V^d(rho) in closed form (Sec. 3.1, eq. for V^0 and the second difference for V^d)
__device__ __forceinline__ double v_closed(const AsmParams &p, double rho, int d) {
  const double ir = 1.0 / rho;
  if (d == 0) return p.kVs * ir - p.kV * (rA_level(p, 1, rho, ir) - rho);
  return p.kV * (2.0 * rA_level(p, d, rho, ir) - rA_level(p, d + 1, rho, ir) -
                 rA_level(p, d - 1, rho, ir));
}

// Per-block Taylor data: the V_h tables (V^{11}) and the odd tables of D^{2,d}, their lengths,
// scales and w factors
struct P1Tabs {
  const double *tscale, *d2tab, *d2scale, *taylor;
  const int32_t *d2len;                 // [nt][2]: D^{2,d} pass lengths, separated and touching
  const int32_t *tlen_sep, *tlen_touch; // [nt]: V_h pass lengths, separated and touching
};

// ---- separated pairs ----
// The task list of the V_h / K_h assembly: one wave per task, test panel l uniform (its rule nodes
// in LDS), up to 64 trial panels m0, m0 + 1, ... (mod E_x), each unordered pair once.  A pair's
// block is S[i][j] = sum_{a, b} w_a w_b lambda_a,i lambda_b,j k(x_a - y_b) (test vertex i of l,
// trial vertex j of m): per trial node b the test-node sums u_i = sum_a w_a lambda_a,i k are
// formed, then weighted by the trial basis.  The closed-form blocks go one per pass, the Taylor
// blocks two per pass sharing r and rho^2.  Contributions to row vl[i] of the workspace W are
// summed per distinct trial vertex of the task in LDS and added to W once per vertex and pass.
struct P1Lane {
  const double *xs;   // LDS [kFarN][4]: test nodes of l and the rule weight
  const double *lam;  // LDS [kFarN][4]: barycentrics of the rule nodes and the weight
  double shift;       // inactive lanes integrate a far-away copy and store nothing
};

template <int KIND>
__device__ __forceinline__ void p1_closed_block(const AsmParams &p, int m, int d, const P1Lane &L,
                                                double S[3][3]) {
  const int ne = p.ne;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = 0.0;
#pragma unroll 1
  for (int b = 0; b < kFarN; ++b) {
    const double y0 = p.geom[(b * 3 + 0) * ne + m] + L.shift;
    const double y1 = p.geom[(b * 3 + 1) * ne + m];
    const double y2 = p.geom[(b * 3 + 2) * ne + m];
    double u[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int a = 0; a < kFarN; ++a) {
      const RuleNode X = rule_node(L.xs, a);
      const double rx = X.x - y0, ry = X.y - y1, rz = X.z - y2;
      const double rho = sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
      const double k = X.w * (KIND == kKindD2 ? d2_closed(p, rho, d) : v_closed(p, rho, d));
      const RuleNode La = rule_node(L.lam, a);
      u[0] = fma(La.x, k, u[0]);
      u[1] = fma(La.y, k, u[1]);
      u[2] = fma(La.z, k, u[2]);
    }
    const RuleNode Lb = rule_node(L.lam, b);
    const double phi[3] = {Lb.w * Lb.x, Lb.w * Lb.y, Lb.w * Lb.z};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) S[i][j] = fma(phi[j], u[i], S[i][j]);
  }
}

// Taylor polynomial, its scale and w factor of block d
template <int KIND>
__device__ __forceinline__ const double *p1_poly(const P1Tabs &T, int d, double &cw, double &sc) {
  cw = T.tscale[3 * d + 2];
  if constexpr (KIND == kKindD2) {
    sc = T.d2scale[d];
    return T.d2tab + (size_t)d * kTaylorND;
  } else {
    sc = T.tscale[3 * d];
    return T.taylor + (size_t)(2 * d) * kTaylorN;
  }
}

// Taylor blocks d0 and d1 (d1 = d0 + 1, or d0 itself at the end) with the polynomial length N of
// block d0 (the tables hold block d1 at that length, or zeros past its own).
template <int KIND, int N>
__device__ __forceinline__ void p1_taylor2(const AsmParams &p, const P1Tabs &T, int d0, int d1,
                                           int m, const P1Lane &L, const double *etab,
                                           double S0[3][3], double S1[3][3]) {
  const int ne = p.ne;
  double cw0, sc0, cw1, sc1;
  const double *c0 = p1_poly<KIND>(T, d0, cw0, sc0);
  const double *c1 = p1_poly<KIND>(T, d1, cw1, sc1);
  // rho^2 clamped where e^{-w} of both blocks is 0 anyway (w >= 1000 for the smaller factor; the
  // larger one is at most (d0 + 1) / d0 times it)
  const double r2max = 1000.0 / fmin(cw0, cw1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S0[i][j] = S1[i][j] = 0.0;
#pragma unroll 1
  for (int b = 0; b < kFarN; ++b) {
    const double y0 = p.geom[(b * 3 + 0) * ne + m] + L.shift;
    const double y1 = p.geom[(b * 3 + 1) * ne + m];
    const double y2 = p.geom[(b * 3 + 2) * ne + m];
    double u0[3] = {0.0, 0.0, 0.0}, u1[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < kFarN; ++a) {
      const RuleNode X = rule_node(L.xs, a);
      const double rx = X.x - y0, ry = X.y - y1, rz = X.z - y2;
      const double rho2 = fmin(fma(rx, rx, fma(ry, ry, rz * rz)), r2max);
      const double w0 = rho2 * cw0, w1 = rho2 * cw1;
      const double k0 = X.w * exp_neg_mu(w0, etab) * horner<N>(c0, w0);
      const double k1 = X.w * exp_neg_mu(w1, etab) * horner<N>(c1, w1);
      const RuleNode La = rule_node(L.lam, a);
      u0[0] = fma(La.x, k0, u0[0]);
      u0[1] = fma(La.y, k0, u0[1]);
      u0[2] = fma(La.z, k0, u0[2]);
      u1[0] = fma(La.x, k1, u1[0]);
      u1[1] = fma(La.y, k1, u1[1]);
      u1[2] = fma(La.z, k1, u1[2]);
    }
    const RuleNode Lb = rule_node(L.lam, b);
    const double phi[3] = {Lb.w * Lb.x, Lb.w * Lb.y, Lb.w * Lb.z};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        S0[i][j] = fma(phi[j], u0[i], S0[i][j]);
        S1[i][j] = fma(phi[j], u1[i], S1[i][j]);
      }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S0[i][j] *= sc0;
      S1[i][j] *= sc1;
    }
}

// Dispatch of a Taylor pass to the polynomial length of its first block.
template <int KIND>
__device__ __forceinline__ void p1_taylor_pass(const AsmParams &p, const P1Tabs &T, int d0, int d1,
                                               int m, const P1Lane &L, const double *etab,
                                               double S0[3][3], double S1[3][3]) {
  if constexpr (KIND == kKindD2) {
    switch (T.d2len[2 * d0]) {  // one of kD2Lens
      case 4: p1_taylor2<KIND, 4>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 6: p1_taylor2<KIND, 6>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 8: p1_taylor2<KIND, 8>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 10: p1_taylor2<KIND, 10>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 12: p1_taylor2<KIND, 12>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 14: p1_taylor2<KIND, 14>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 16: p1_taylor2<KIND, 16>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 20: p1_taylor2<KIND, 20>(p, T, d0, d1, m, L, etab, S0, S1); break;
      default: p1_taylor2<KIND, 24>(p, T, d0, d1, m, L, etab, S0, S1); break;
    }
  } else {
    switch (T.tlen_sep[d0]) {  // one of kPolyLens
      case 5: p1_taylor2<KIND, 5>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 6: p1_taylor2<KIND, 6>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 7: p1_taylor2<KIND, 7>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 8: p1_taylor2<KIND, 8>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 9: p1_taylor2<KIND, 9>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 10: p1_taylor2<KIND, 10>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 11: p1_taylor2<KIND, 11>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 13: p1_taylor2<KIND, 13>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 15: p1_taylor2<KIND, 15>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 17: p1_taylor2<KIND, 17>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 19: p1_taylor2<KIND, 19>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 21: p1_taylor2<KIND, 21>(p, T, d0, d1, m, L, etab, S0, S1); break;
      case 25: p1_taylor2<KIND, 25>(p, T, d0, d1, m, L, etab, S0, S1); break;
      default: p1_taylor2<KIND, 29>(p, T, d0, d1, m, L, etab, S0, S1); break;
    }
  }
}

template <int KIND, typename TS>
__global__ __launch_bounds__(256, 2) void k_p1_separated(const AsmParams *__restrict__ pp, P1Tabs T,
                                                         const int32_t *__restrict__ tasks,
                                                         const int *__restrict__ tvstart,
                                                         const int *__restrict__ tverts,
                                                         const uint8_t *__restrict__ tslots,
                                                         int ntasks, TS *__restrict__ W) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  __shared__ double lam[kFarN * 4];
  __shared__ double xs[4][kFarN * 4];
  // the pass's contributions (up to two blocks) to rows vl[0..2] per distinct trial vertex
  __shared__ double wacc[4][2][3][kSepSlots];
  stage_exp_tab_pos(etab);
  const int task = xcd_block() * 4 + (threadIdx.x >> 6);
  const bool valid = task < ntasks;
  const int l = valid ? __builtin_amdgcn_readfirstlane(tasks[3 * task]) : 0;
  stage_test_nodes(p, p.geom, l, valid, xs[threadIdx.x >> 6], lam);
  __syncthreads();
  if (!valid) return;
  const int lane = threadIdx.x & 63;
  // lanes past the task's count integrate a copy of its first pair and store nothing (they stay
  // for the per-vertex flush)
  const bool inrange = lane < __builtin_amdgcn_readfirstlane(tasks[3 * task + 2]);
  const int ne = p.ne, nv = p.nv;
  int m = __builtin_amdgcn_readfirstlane(tasks[3 * task + 1]) + (inrange ? lane : 0);
  if (m >= ne) m -= ne;
  const int vl[3] = {p.tris[3 * l], p.tris[3 * l + 1], p.tris[3 * l + 2]};
  const int vm[3] = {p.tris[3 * m], p.tris[3 * m + 1], p.tris[3 * m + 2]};
  bool touch = false;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) touch |= vl[i] == vm[j];  // touching: the regularised rules
  const bool active = inrange && !touch;
  double(*acc)[3][kSepSlots] = wacc[threadIdx.x >> 6];
  const int sv0 = __builtin_amdgcn_readfirstlane(tvstart[task]);
  const int nslots = __builtin_amdgcn_readfirstlane(tvstart[task + 1]) - sv0;
  int slot[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) slot[k] = tslots[((size_t)task * 3 + k) * 64 + lane];
  for (int e = lane; e < 2 * 3 * kSepSlots; e += 64) (&acc[0][0][0])[e] = 0.0;
  wave_lds_sync();
  const double nn = KIND == kKindD2 ? p.geom[21 * ne + l] * p.geom[21 * ne + m] +
                                          p.geom[22 * ne + l] * p.geom[22 * ne + m] +
                                          p.geom[23 * ne + l] * p.geom[23 * ne + m]
                                    : 1.0;
  const double scale = nn * p.geom[24 * ne + l] * p.geom[24 * ne + m];
  P1Lane L{xs[threadIdx.x >> 6], lam, active ? 0.0 : 1.0e3};
  // blocks [d, d + nb) of this pass into LDS, then each vertex's sums to W once
  auto emit = [&](int d, int nb, double S0[3][3], double S1[3][3]) {
    if (active) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          atomicAdd(&acc[0][i][slot[k]], scale * S0[i][k]);
          if (nb > 1) atomicAdd(&acc[1][i][slot[k]], scale * S1[i][k]);
        }
    }
    wave_lds_sync();
    for (int sidx = lane; sidx < nslots; sidx += 64) {
      const int v = tverts[sv0 + sidx];
      for (int j = 0; j < nb; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double a = acc[j][i][sidx];
          if (a != 0.0) atomicAdd(&W[((size_t)(d + j) * nv + vl[i]) * nv + v], (TS)a);
          acc[j][i][sidx] = 0.0;
        }
    }
    wave_lds_sync();
  };
  const int nclosed = KIND == kKindD2 ? min(kD2Closed, p.nt) : min(p.dsw, p.nt);
  for (int d = 0; d < nclosed; ++d) {
    double S[3][3];
    p1_closed_block<KIND>(p, m, d, L, S);
    emit(d, 1, S, S);
  }
  for (int d = nclosed; d < p.nt; d += 2) {
    double S0[3][3], S1[3][3];
    const int d1 = min(d + 1, p.nt - 1);
    p1_taylor_pass<KIND>(p, T, d, d1, m, L, etab, S0, S1);
    emit(d, d1 > d ? 2 : 1, S0, S1);
  }
}

// D[d] = W[d] + W[d]^T, 64 x 64 tiles through LDS
template <typename TS>
__global__ __launch_bounds__(256) void k_sym_blocks(const TS *__restrict__ W, TS *__restrict__ D, int n) {
  __shared__ TS tile[64][65];
  const size_t off = (size_t)blockIdx.z * n * n;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // tile of W^T: rows j0.., columns i0.. of W
  for (int r = ty; r < 64; r += 4) {
    const int row = j0 + r, col = i0 + tx;
    tile[r][tx] = (row < n && col < n) ? W[off + (size_t)row * n + col] : TS(0);
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int row = i0 + r, col = j0 + tx;
    if (row < n && col < n) D[off + (size_t)row * n + col] = W[off + (size_t)row * n + col] + tile[tx][r];
  }
}

// ---- touching pairs ----
// One wave per list entry: identical and edge-sharing pairs per ordered pair, vertex-sharing pairs
// once for both orders (SYM: their rule serves the swapped pair with test and trial exchanged, so
// the block of the order (m, l) is the transpose).  Lanes stride over the rule points; blocks go
// one per pass in closed form, two per pass in Taylor form.  The pass's 18 sums (two blocks x 3
// test x 3 trial vertices) leave the lanes through LDS: row i holds the 64 partial sums of sum i,
// lanes 2 i and 2 i + 1 add its halves and lane 2 i stores it.
constexpr int kP1Sums = 18;
constexpr int kP1RedRow = 66;  // LDS row of one sum's partial sums (padded against bank conflicts)

template <int KIND, int N>  // N = 0: block d0 in closed form (d1 unused)
__device__ __forceinline__ void p1_touch_pass(const AsmParams &p, const P1Tabs &T,
                                              const TouchPair &tp, const RuleCols &col, int cls,
                                              int ntab, int d0, int d1, const double *etab,
                                              double R[kP1Sums]) {
  double cw0 = 0.0, sc0 = 1.0, cw1 = 0.0, sc1 = 1.0, r2max = 0.0;
  const double *c0 = nullptr, *c1 = nullptr;
  if constexpr (N > 0) {
    c0 = p1_poly<KIND>(T, d0, cw0, sc0);
    c1 = p1_poly<KIND>(T, d1, cw1, sc1);
    r2max = 1000.0 / fmin(cw0, cw1);
  }
#pragma unroll
  for (int i = 0; i < kP1Sums; ++i) R[i] = 0.0;
#pragma unroll 1
  for (int q = threadIdx.x; q < ntab; q += 64) {
    const unsigned off = 8u * q;
    // (cls is uniform) the vertex rule stores the reference coordinates c = (x1, x2, -y1, -y2),
    // from which both barycentric triples follow; the identical rule's third and fourth and the
    // edge rule's third coordinate are zero, and the edge rule's fourth is -y2
    const double a1 = col.at(0, off), a2 = col.at(1, off);
    const double a3 = cls == 1 ? col.at(2, off) : 0.0, a4 = cls == 3 ? 0.0 : col.at(3, off);
    const double rx = a1 * tp.E1[0] + a2 * tp.E2[0] + a3 * tp.F1[0] + a4 * tp.F2[0];
    const double ry = a1 * tp.E1[1] + a2 * tp.E2[1] + a3 * tp.F1[1] + a4 * tp.F2[1];
    const double rz = a1 * tp.E1[2] + a2 * tp.E2[2] + a3 * tp.F1[2] + a4 * tp.F2[2];
    const double rho2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const double W = col.at(4, off);
    double ly[3], lx[3];
    if (cls == 1) {
      ly[0] = 1.0 + a3;
      ly[1] = a4 - a3;
      ly[2] = -a4;
      lx[0] = 1.0 - a1;
      lx[1] = a1 - a2;
      lx[2] = a2;
    } else {
      ly[0] = col.at(5, off);
      ly[1] = col.at(6, off);
      ly[2] = cls == 2 ? -a4 : col.at(7, off);
      lx[0] = col.at(8, off);
      lx[1] = col.at(9, off);
      lx[2] = col.at(10, off);
    }
    double k0, k1 = 0.0;
    if constexpr (N == 0) {
      const double rho = sqrt(rho2);
      k0 = W * (KIND == kKindD2 ? d2_closed(p, rho, d0) : v_closed(p, rho, d0));
    } else {
      const double r2 = fmin(rho2, r2max);
      const double w0 = r2 * cw0, w1 = r2 * cw1;
      k0 = W * exp_neg_mu(w0, etab) * horner<N>(c0, w0);
      k1 = W * exp_neg_mu(w1, etab) * horner<N>(c1, w1);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u0 = k0 * lx[i], u1 = k1 * lx[i];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        R[3 * i + k] = fma(u0, ly[k], R[3 * i + k]);
        if constexpr (N > 0) R[9 + 3 * i + k] = fma(u1, ly[k], R[9 + 3 * i + k]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    R[i] *= sc0;
    R[9 + i] *= sc1;
  }
}

// Dispatch of a pass to the polynomial length of its first block (0: closed form).
template <int KIND>
__device__ __forceinline__ void p1_touch_dispatch(const AsmParams &p, const P1Tabs &T,
                                                  const TouchPair &tp, const RuleCols &col,
                                                  int cls, int ntab, int len, int d0, int d1,
                                                  const double *etab, double R[kP1Sums]) {
  if constexpr (KIND == kKindD2) {
    switch (len) {  // 0 or one of kD2Lens
      case 0: p1_touch_pass<KIND, 0>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 4: p1_touch_pass<KIND, 4>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 6: p1_touch_pass<KIND, 6>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 8: p1_touch_pass<KIND, 8>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 10: p1_touch_pass<KIND, 10>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 12: p1_touch_pass<KIND, 12>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 14: p1_touch_pass<KIND, 14>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 16: p1_touch_pass<KIND, 16>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 20: p1_touch_pass<KIND, 20>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      default: p1_touch_pass<KIND, 24>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
    }
  } else {
    switch (len) {  // 0 or one of kPolyLens
      case 0: p1_touch_pass<KIND, 0>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 5: p1_touch_pass<KIND, 5>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 6: p1_touch_pass<KIND, 6>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 7: p1_touch_pass<KIND, 7>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 8: p1_touch_pass<KIND, 8>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 9: p1_touch_pass<KIND, 9>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 10: p1_touch_pass<KIND, 10>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 11: p1_touch_pass<KIND, 11>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 13: p1_touch_pass<KIND, 13>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 15: p1_touch_pass<KIND, 15>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 17: p1_touch_pass<KIND, 17>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 19: p1_touch_pass<KIND, 19>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 21: p1_touch_pass<KIND, 21>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      case 25: p1_touch_pass<KIND, 25>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
      default: p1_touch_pass<KIND, 29>(p, T, tp, col, cls, ntab, d0, d1, etab, R); break;
    }
  }
}

// One list entry (a wave): ent indexes pairs (SYM: ~index of a vertex pair, both orders).
template <int KIND, typename TS, bool SYM>
__device__ __forceinline__ void p1_touch_entry(const AsmParams &p,
                                               const TouchPair *__restrict__ pairs, int ent,
                                               const RuleTabs &rules, const P1Tabs &T,
                                               TS *__restrict__ D, const double *etab,
                                               double *red) {
  const TouchPair &tp = pairs[SYM ? ~ent : ent];
  const int cls = __builtin_amdgcn_readfirstlane(tp.cls);
  const int ntab = rules.n[cls];
  const RuleCols col(rules.d[cls], ntab);
  const int lane = threadIdx.x, nv = p.nv;
  const double f = tp.scale * (KIND == kKindD2 ? tp.nn : 1.0);
  // the sum this lane stores: lane 2 i, sum i = (block j, test vertex ii, trial vertex kk)
  const int si = lane >> 1, sj = si / 9, sii = (si % 9) / 3, skk = si % 3;
  const bool mine = (lane & 1) == 0 && si < kP1Sums;
  const int drow = mine ? tp.vtxl[sii] : 0, dcol = mine ? tp.vtx[skk] : 0;
  const int nclosed = KIND == kKindD2 ? min(kD2Closed, p.nt) : min(p.dsw, p.nt);
  for (int d = 0; d < p.nt;) {
    const bool closed = d < nclosed;
    const int d1 = closed ? d : min(d + 1, p.nt - 1);
    const int nb = closed || d1 == d ? 1 : 2;
    const int len = closed ? 0 : (KIND == kKindD2 ? T.d2len[2 * d + 1] : T.tlen_touch[d]);
    double R[kP1Sums];
    p1_touch_dispatch<KIND>(p, T, tp, col, cls, ntab, len, d, d1, etab, R);
#pragma unroll
    for (int i = 0; i < kP1Sums; ++i) red[i * kP1RedRow + lane] = R[i];
    __syncthreads();
    double v = 0.0;
    if (si < kP1Sums) {
      const double *q = red + si * kP1RedRow + 32 * (lane & 1);
#pragma unroll
      for (int k = 0; k < 32; k += 2) {
        const double2 a = *(const double2 *)(q + k);
        v += a.x + a.y;
      }
    }
    v += dpp_d<0xB1>(v);  // quad_perm [1, 0, 3, 2]: the two halves
    __syncthreads();
    if (mine && sj < nb) {
      TS *Dd = D + (size_t)(d + sj) * nv * nv;
      atomicAdd(&Dd[(size_t)drow * nv + dcol], (TS)(f * v));
      if constexpr (SYM) atomicAdd(&Dd[(size_t)dcol * nv + drow], (TS)(f * v));
    }
    d += nb;
  }
}

// All touching pairs in one launch: the first n0 list entries one order each (identical and edge
// pairs, the longest rules first), the rest vertex pairs for both orders.
template <int KIND, typename TS>
__global__ __launch_bounds__(64, 3) void k_p1_touching(const AsmParams *__restrict__ pp,
                                                       const TouchPair *__restrict__ pairs,
                                                       const int32_t *__restrict__ list, int n0,
                                                       RuleTabs rules, P1Tabs T,
                                                       TS *__restrict__ D) {
  const AsmParams &p = *pp;
  __shared__ double etab[kExpTabN];
  __shared__ __align__(16) double red[kP1Sums * kP1RedRow];
  stage_exp_tab_pos(etab);
  __syncthreads();
  const int ent = __builtin_amdgcn_readfirstlane(list[blockIdx.x]);
  if ((int)blockIdx.x < n0)
    p1_touch_entry<KIND, TS, false>(p, pairs, ent, rules, T, D, etab, red);
  else
    p1_touch_entry<KIND, TS, true>(p, pairs, ent, rules, T, D, etab, red);
}

// D[d][i][j] += alpha^2 sum_{(n, a) at i} sum_{(m, b) at j} curl_a(n) . curl_b(m) V[d][n][m]
// One thread per j, one workgroup per (i, d): the panels at j and their curls are loaded once
// (kD1Chunk at a time, in registers), then each panel n at i (uniform) meets them all.
constexpr int kD1Chunk = 8;

template <typename TS>
__global__ __launch_bounds__(256) void k_d1(const TS *__restrict__ V, TS *__restrict__ D,
                                            const double *__restrict__ curl,
                                            const int32_t *__restrict__ vstart,
                                            const int32_t *__restrict__ vadj, int ne, int nv,
                                            double a2) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y, d = blockIdx.z;
  if (j >= nv) return;
  const TS *Vd = V + (size_t)d * ne * ne;
  const int i0 = vstart[i], i1 = vstart[i + 1], j0 = vstart[j], j1 = vstart[j + 1];
  double acc = 0.0;
  for (int t0 = j0; t0 < j1; t0 += kD1Chunk) {
    int mm[kD1Chunk];
    double cx[kD1Chunk], cy[kD1Chunk], cz[kD1Chunk];
#pragma unroll
    for (int u = 0; u < kD1Chunk; ++u) {
      const bool in = t0 + u < j1;
      const int m = in ? vadj[2 * (t0 + u)] : 0, b = in ? vadj[2 * (t0 + u) + 1] : 0;
      mm[u] = m;
      cx[u] = in ? curl[9 * m + 3 * b] : 0.0;  // zero curls: the padding adds nothing
      cy[u] = in ? curl[9 * m + 3 * b + 1] : 0.0;
      cz[u] = in ? curl[9 * m + 3 * b + 2] : 0.0;
    }
    for (int s = i0; s < i1; ++s) {
      const int n = vadj[2 * s], a = vadj[2 * s + 1];
      const double c0 = curl[9 * n + 3 * a], c1 = curl[9 * n + 3 * a + 1], c2 = curl[9 * n + 3 * a + 2];
      const TS *row = Vd + (size_t)n * ne;
#pragma unroll
      for (int u = 0; u < kD1Chunk; ++u)
        acc = fma(fma(c0, cx[u], fma(c1, cy[u], c2 * cz[u])), (double)row[mm[u]], acc);
    }
  }
  TS *out = D + ((size_t)d * nv + i) * nv + j;
  *out = (TS)((double)*out + a2 * acc);
}

// dst[d] = src[d]^T for blocks [nt][R][C], 64 x 64 tiles through LDS
template <typename TS>
__global__ __launch_bounds__(256) void k_transpose_blocks(const TS *__restrict__ src,
                                                          TS *__restrict__ dst, int R, int C) {
  __shared__ TS tile[64][65];
  const size_t off = (size_t)blockIdx.z * R * C;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int row = r0 + r, col = c0 + tx;
    if (row < R && col < C) tile[r][tx] = src[off + (size_t)row * C + col];
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int row = c0 + r, col = r0 + tx;  // dst is C x R
    if (row < C && col < R) dst[off + (size_t)row * R + col] = tile[tx][r];
  }
}

// p1 x p1 blocks of kind KIND into out: separated pairs into the workspace, out = W + W^T, then
// the touching pairs
template <int KIND, typename TS>
int assemble_p1p1(hb_ctx *c, TS *out, hipStream_t s) {
  const int nt = c->nt, nv = (int)c->nv;
  const size_t nD = (size_t)nt * nv * nv;
  TS *W = (TS *)c->d_Dw;
  P1Tabs T{c->d_tscale, c->d_d2tab, c->d_d2scale, c->d_taylor, c->d_d2len, c->d_tlen_sep,
           c->d_tlen_touch};
  if (hipMemsetAsync(W, 0, nD * sizeof(TS), s) != hipSuccess) return HB_EHIP;
  if (c->n_sep_tasks > 0)
    hipLaunchKernelGGL((k_p1_separated<KIND, TS>), dim3((unsigned)((c->n_sep_tasks + 3) / 4)),
                       dim3(256), 0, s, c->d_params, T, c->d_sep_tasks, c->d_sep_vstart,
                       c->d_sep_verts, c->d_sep_slots, (int)c->n_sep_tasks, W);
  const dim3 tiles((nv + 63) / 64, (nv + 63) / 64, nt);
  hipLaunchKernelGGL((k_sym_blocks<TS>), tiles, dim3(256), 0, s, W, out, nv);
  if (c->n_touch_list > 0) {
    RuleTabs rt{};
    for (int k = 1; k <= 3; ++k) {
      rt.d[k] = c->ss[k].d;
      rt.n[k] = c->ss[k].n;
    }
    // the touching list: identical and edge pairs of both orders, then the vertex pairs once
    const int nsym = (int)c->n_touch_sym, n0 = (int)c->n_touch_list - nsym;
    hipLaunchKernelGGL((k_p1_touching<KIND, TS>), dim3((unsigned)c->n_touch_list), dim3(64), 0, s,
                       c->d_params, c->d_touch, c->d_touch_list, n0, rt, T, out);
  }
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

template <typename TS>
int assemble_d_typed(hb_ctx *c, hipStream_t s) {
  const int nt = c->nt, ne = (int)c->ne, nv = (int)c->nv;
  TS *D = (TS *)c->d_D;
  int rc = assemble_p1p1<kKindD2, TS>(c, D, s);
  if (rc) return rc;
  hipLaunchKernelGGL((k_d1<TS>), dim3((nv + 255) / 256, nv, nt), dim3(256), 0, s,
                     (const TS *)c->d_V, D, c->d_curl, c->d_vstart, c->d_vadj, ne, nv,
                     c->alpha * c->alpha);
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

template <typename TS>
void transpose_typed(const void *src, void *dst, int R, int C, int nt, hipStream_t s) {
  hipLaunchKernelGGL((k_transpose_blocks<TS>), dim3((C + 63) / 64, (R + 63) / 64, nt), dim3(256),
                     0, s, (const TS *)src, (TS *)dst, R, C);
}

}  // namespace

int launch_assemble_d(hb_ctx *c, hipStream_t s) {
  return c->storage_f32 ? assemble_d_typed<float>(c, s) : assemble_d_typed<double>(c, s);
}

int launch_assemble_v11(hb_ctx *c, hipStream_t s) {
  return c->storage_f32 ? assemble_p1p1<kKindV11, float>(c, (float *)c->d_V11, s)
                        : assemble_p1p1<kKindV11, double>(c, (double *)c->d_V11, s);
}

int launch_transpose_blocks(hb_ctx *c, const void *src, void *dst, int R, int C, hipStream_t s) {
  if (c->storage_f32) transpose_typed<float>(src, dst, R, C, c->nt, s);
  else transpose_typed<double>(src, dst, R, C, c->nt, s);
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

}  // namespace hb
