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
// trial panels, each unordered pair once), Radon's rule on both panels, contributions added to the workspace row block of l; then
// D^2 = W + W^T.  Touching pairs: one wave per ordered pair, the regularised rule of its class.
// D_h^{1,d} = T^T (alpha^2 V^d (x) I_3) T (Sec. 3.3, eq. for D_h^{1,d}) is added entry by entry
// from V_h^d and the surface curls of the local p1 basis.
// The same p1 x p1 kernels assemble V_h^{11}, the single layer between p1 functions (the matrix
// of the paper's preconditioner for D_h, Sec. 6.1), with the kernel V^d(r) of V_h: closed form
// (second differences of G^{dtau dt} = rho A(z) / (8 pi alpha^2)) below d_switch, the even Taylor
// tables of V_h above, and no normal factor.
#include "hb_closed.h"
#include "hb_device.h"
#include "hb_internal.h"

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

// Kernel value at rho^2 for block d (N = 0: closed form; else the Taylor polynomial with N
// coefficients, scale sc, w = rho^2 cw)
template <int KIND, int N>
__device__ __forceinline__ double kern_value(const AsmParams &p, double rho2, int d, double ah,
                                             double cw, double sc, const double *__restrict__ tab,
                                             const double *etab) {
  if constexpr (N == 0) {
    if constexpr (KIND == kKindD2) return d2_closed(p, sqrt(rho2), d);
    else return v_closed(p, sqrt(rho2), d);
  } else {
    const double w = rho2 * cw;
    return sc * exp_neg_t(w, etab) * horner<N>(tab, w);
  }
}

// Per-block Taylor data of kind KIND: polynomial, its length, scale and w factor
struct P1Tabs {
  const double *tscale, *d2tab, *d2scale, *taylor;
  const int32_t *d2len, *tdeg;
};

template <int KIND>
__device__ __forceinline__ int block_len(const AsmParams &p, const P1Tabs &T, int d) {
  if constexpr (KIND == kKindD2) return d < kD2Closed ? 0 : T.d2len[d];
  else return d < p.dsw ? 0 : T.tdeg[2 * d] + 1;
}

template <int KIND>
__device__ __forceinline__ void block_tab(const P1Tabs &T, int d, double &cw, double &sc,
                                          const double *&tab) {
  cw = T.tscale[3 * d + 2];
  if constexpr (KIND == kKindD2) {
    sc = T.d2scale[d];
    tab = T.d2tab + (size_t)d * kTaylorND;
  } else {
    sc = T.tscale[3 * d];
    tab = T.taylor + (size_t)(2 * d) * kTaylorN;
  }
}

// One block d of a separated pair: S[a][b] = sum over the 7 x 7 point pairs of the weights, the
// kernel and the test / trial barycentrics.
template <int KIND, int N>
__device__ __forceinline__ void p1_sep_block(const AsmParams &p, int l, int m, int d, double ah,
                                             const P1Tabs &T, const double *etab, double S[3][3]) {
  const int ne = p.ne;
  double cw = 0.0, sc = 0.0;
  const double *tab = nullptr;
  if constexpr (N > 0) block_tab<KIND>(T, d, cw, sc, tab);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = 0.0;
#pragma unroll 1
  for (int a = 0; a < kFarN; ++a) {
    const double x0 = p.geom[(a * 3 + 0) * ne + l], x1 = p.geom[(a * 3 + 1) * ne + l],
                 x2 = p.geom[(a * 3 + 2) * ne + l];
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll 1
    for (int b = 0; b < kFarN; ++b) {
      const double rx = x0 - p.geom[(b * 3 + 0) * ne + m];
      const double ry = x1 - p.geom[(b * 3 + 1) * ne + m];
      const double rz = x2 - p.geom[(b * 3 + 2) * ne + m];
      const double v = p.w7[b] * kern_value<KIND, N>(p, fma(rx, rx, fma(ry, ry, rz * rz)), d, ah, cw, sc, tab, etab);
      t0 = fma(v, p.lam7[b][0], t0);
      t1 = fma(v, p.lam7[b][1], t1);
      t2 = fma(v, p.lam7[b][2], t2);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double wa = p.w7[a] * p.lam7[a][i];
      S[i][0] = fma(wa, t0, S[i][0]);
      S[i][1] = fma(wa, t1, S[i][1]);
      S[i][2] = fma(wa, t2, S[i][2]);
    }
  }
}

// One block of a separated / touching pair as a functor templated on the polynomial length.
template <int KIND>
struct SepBlock {
  const AsmParams &p;
  int l, m, d;
  double ah;
  const P1Tabs &T;
  const double *etab;
  double (&S)[3][3];
  template <int N>
  __device__ __forceinline__ void operator()() const {
    p1_sep_block<KIND, N>(p, l, m, d, ah, T, etab, S);
  }
};

template <int KIND, int N>
__device__ __forceinline__ void p1_touch_block(const AsmParams &p, const TouchPair &tp,
                                               const double *__restrict__ tab, int ntab, int lane,
                                               int d, double ah, const P1Tabs &T,
                                               const double *etab, double S[9]);

template <int KIND>
struct TouchBlock {
  const AsmParams &p;
  const TouchPair &tp;
  const double *tab;
  int ntab, lane, d;
  double ah;
  const P1Tabs &T;
  const double *etab;
  double (&S)[9];
  template <int N>
  __device__ __forceinline__ void operator()() const {
    p1_touch_block<KIND, N>(p, tp, tab, ntab, lane, d, ah, T, etab, S);
  }
};

// Dispatch of one block to the polynomial length of its table (0: closed form).
template <int KIND, typename F>
__device__ __forceinline__ void by_len(int len, F &&f) {
  switch (len) {
    case 0: f.template operator()<0>(); break;
    case 29: if constexpr (KIND == kKindV11) f.template operator()<29>(); break;
    case 25: if constexpr (KIND == kKindV11) f.template operator()<25>(); break;
    case 21: if constexpr (KIND == kKindV11) f.template operator()<21>(); break;
    case 19: if constexpr (KIND == kKindV11) f.template operator()<19>(); break;
    case 17: if constexpr (KIND == kKindV11) f.template operator()<17>(); break;
    case 16: if constexpr (KIND == kKindD2) f.template operator()<16>(); break;
    case 15: if constexpr (KIND == kKindV11) f.template operator()<15>(); break;
    case 14: if constexpr (KIND == kKindD2) f.template operator()<14>(); break;
    case 13: if constexpr (KIND == kKindV11) f.template operator()<13>(); break;
    case 12: if constexpr (KIND == kKindD2) f.template operator()<12>(); break;
    case 11: if constexpr (KIND == kKindV11) f.template operator()<11>(); break;
    case 10: if constexpr (KIND == kKindD2) f.template operator()<10>(); break;
    case 9: if constexpr (KIND == kKindV11) f.template operator()<9>(); break;
    case 8: if constexpr (KIND == kKindD2) f.template operator()<8>(); break;
    default: if constexpr (KIND == kKindV11) f.template operator()<7>(); break;
  }
}

template <int KIND, typename TS>
__global__ __launch_bounds__(256) void k_p1_separated(const AsmParams *__restrict__ pp, P1Tabs T,
                                                      const int32_t *__restrict__ tasks,
                                                      int ntasks, TS *__restrict__ W) {
  const AsmParams &p = *pp;
  __shared__ double etab[64];
  stage_exp_tab(etab);
  __syncthreads();
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= ntasks) return;
  const int l = __builtin_amdgcn_readfirstlane(tasks[3 * task]);
  const int lane = threadIdx.x & 63;
  if (lane >= __builtin_amdgcn_readfirstlane(tasks[3 * task + 2])) return;
  const int ne = p.ne, nv = p.nv;
  int m = __builtin_amdgcn_readfirstlane(tasks[3 * task + 1]) + lane;
  if (m >= ne) m -= ne;
  const int vl[3] = {p.tris[3 * l], p.tris[3 * l + 1], p.tris[3 * l + 2]};
  const int vm[3] = {p.tris[3 * m], p.tris[3 * m + 1], p.tris[3 * m + 2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (vl[i] == vm[j]) return;  // touching: handled by the regularised rules
  const double nn = KIND == kKindD2 ? p.geom[21 * ne + l] * p.geom[21 * ne + m] +
                                          p.geom[22 * ne + l] * p.geom[22 * ne + m] +
                                          p.geom[23 * ne + l] * p.geom[23 * ne + m]
                                    : 1.0;
  const double scale = nn * p.geom[24 * ne + l] * p.geom[24 * ne + m];
  const double ah = p.alpha * p.h;
  for (int d = 0; d < p.nt; ++d) {
    double S[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    by_len<KIND>(block_len<KIND>(p, T, d), SepBlock<KIND>{p, l, m, d, ah, T, etab, S});
    TS *Wb = W + (size_t)d * nv * nv;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) atomicAdd(&Wb[(size_t)vl[i] * nv + vm[j]], (TS)(scale * S[i][j]));
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

template <int KIND, int N>
__device__ __forceinline__ void p1_touch_block(const AsmParams &p, const TouchPair &tp,
                                               const double *__restrict__ tab, int ntab, int lane,
                                               int d, double ah, const P1Tabs &T,
                                               const double *etab, double S[9]) {
  double cw = 0.0, sc = 0.0;
  const double *poly = nullptr;
  if constexpr (N > 0) block_tab<KIND>(T, d, cw, sc, poly);
#pragma unroll
  for (int k = 0; k < 9; ++k) S[k] = 0.0;
#pragma unroll 1
  for (int q = lane; q < ntab; q += 64) {
    const double a1 = tab[q], a2 = tab[ntab + q], a3 = tab[2 * ntab + q], a4 = tab[3 * ntab + q];
    const double rx = a1 * tp.E1[0] + a2 * tp.E2[0] + a3 * tp.F1[0] + a4 * tp.F2[0];
    const double ry = a1 * tp.E1[1] + a2 * tp.E2[1] + a3 * tp.F1[1] + a4 * tp.F2[1];
    const double rz = a1 * tp.E1[2] + a2 * tp.E2[2] + a3 * tp.F1[2] + a4 * tp.F2[2];
    const double v = tab[4 * ntab + q] *
                     kern_value<KIND, N>(p, fma(rx, rx, fma(ry, ry, rz * rz)), d, ah, cw, sc, poly, etab);
    const double ly0 = tab[5 * ntab + q], ly1 = tab[6 * ntab + q], ly2 = tab[7 * ntab + q];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u = v * tab[(8 + i) * ntab + q];
      S[3 * i + 0] = fma(u, ly0, S[3 * i + 0]);
      S[3 * i + 1] = fma(u, ly1, S[3 * i + 1]);
      S[3 * i + 2] = fma(u, ly2, S[3 * i + 2]);
    }
  }
}

template <int KIND, typename TS>
__global__ __launch_bounds__(64) void k_p1_touching(const AsmParams *__restrict__ pp,
                                                    const TouchPair *__restrict__ pairs,
                                                    RuleTabs rules, P1Tabs T, TS *__restrict__ D) {
  const AsmParams &p = *pp;
  __shared__ double etab[64];
  stage_exp_tab(etab);
  __syncthreads();
  const TouchPair &tp = pairs[blockIdx.x];
  const int cls = __builtin_amdgcn_readfirstlane(tp.cls);
  const double *__restrict__ tab = rules.d[cls];
  const int ntab = rules.n[cls];
  const int lane = threadIdx.x, nv = p.nv;
  const double ah = p.alpha * p.h, f = tp.scale * (KIND == kKindD2 ? tp.nn : 1.0);
  for (int d = 0; d < p.nt; ++d) {
    double S[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    by_len<KIND>(block_len<KIND>(p, T, d), TouchBlock<KIND>{p, tp, tab, ntab, lane, d, ah, T, etab, S});
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) S[k] += __shfl_xor(S[k], o, 64);
    if (lane < 9) {
      double v = S[0];
#pragma unroll
      for (int k = 1; k < 9; ++k)
        if (lane == k) v = S[k];
      atomicAdd(&D[((size_t)d * nv + tp.vtxl[lane / 3]) * nv + tp.vtx[lane % 3]], (TS)(f * v));
    }
  }
}

// D[d][i][j] += alpha^2 sum_{(n, a) at i} sum_{(m, b) at j} curl_a(n) . curl_b(m) V[d][n][m]
template <typename TS>
__global__ __launch_bounds__(256) void k_d1(const TS *__restrict__ V, TS *__restrict__ D,
                                            const double *__restrict__ curl,
                                            const int32_t *__restrict__ vstart,
                                            const int32_t *__restrict__ vadj, int ne, int nv,
                                            double a2) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y, d = blockIdx.z;
  if (j >= nv) return;
  const TS *Vd = V + (size_t)d * ne * ne;
  const int j0 = vstart[j], j1 = vstart[j + 1];
  double acc = 0.0;
  for (int s = vstart[i]; s < vstart[i + 1]; ++s) {
    const int n = vadj[2 * s], a = vadj[2 * s + 1];
    const double c0 = curl[9 * n + 3 * a], c1 = curl[9 * n + 3 * a + 1], c2 = curl[9 * n + 3 * a + 2];
    const TS *row = Vd + (size_t)n * ne;
    for (int t = j0; t < j1; ++t) {
      const int m = vadj[2 * t], b = vadj[2 * t + 1];
      const double dot = c0 * curl[9 * m + 3 * b] + c1 * curl[9 * m + 3 * b + 1] + c2 * curl[9 * m + 3 * b + 2];
      acc = fma(dot, (double)row[m], acc);
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
  P1Tabs T{c->d_tscale, c->d_d2tab, c->d_d2scale, c->d_taylor, c->d_d2len, c->d_tdeg};
  if (hipMemsetAsync(W, 0, nD * sizeof(TS), s) != hipSuccess) return HB_EHIP;
  if (c->n_sep_tasks > 0)
    hipLaunchKernelGGL((k_p1_separated<KIND, TS>), dim3((unsigned)((c->n_sep_tasks + 3) / 4)),
                       dim3(256), 0, s, c->d_params, T, c->d_sep_tasks, (int)c->n_sep_tasks, W);
  const dim3 tiles((nv + 63) / 64, (nv + 63) / 64, nt);
  hipLaunchKernelGGL((k_sym_blocks<TS>), tiles, dim3(256), 0, s, W, out, nv);
  if (!c->touch.empty()) {
    RuleTabs rt{};
    for (int k = 1; k <= 3; ++k) {
      rt.d[k] = c->ss[k].d;
      rt.n[k] = c->ss[k].n;
    }
    hipLaunchKernelGGL((k_p1_touching<KIND, TS>), dim3((unsigned)c->touch.size()), dim3(64), 0, s,
                       c->d_params, c->d_touch, rt, T, out);
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
