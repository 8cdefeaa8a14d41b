// Learned preconditioner for V_h w = b: a sparse approximate inverse M ~ (V_h^0)^{-1} on the
// touching-panel pattern of every row, predicted by a small MLP from local data, applied as a
// block-diagonal right preconditioner (the same M in every time step).
//
// Kernels: the row pattern and its features, the per-row normal equations of the sparse
// approximate inverse (training data), a 3-layer tanh MLP (forward, backward, Adam), the
// quadratic training loss, installation of M and its application.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "hb_internal.h"

namespace hb {
namespace {

#define HB_CHECK_L(ctx, call)                                                             \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      if (ctx) (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return e_ == hipErrorOutOfMemory ? HB_ENOMEM : HB_EHIP;                             \
    }                                                                                     \
  } while (0)

constexpr int S = HB_PC_SLOTS;  // pattern slots per row

inline int grid_for(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 8192); }

// ---------------------------------------------------------------------------------------------
// Features of row l (HB_PC_FEATURES floats): per slot s (HB_PC_SLOT_FEATURES each)
//   V^0[l, m_s] / V^0[l, l], one-hot of the pair class (identical, edge, vertex),
//   |c_l - c_m| / sqrt(area_l), area_m / area_l, n_l . n_m, slot present;
// then sqrt(alpha h / area_l), log of it, (number of slots) / S, 1.
// ---------------------------------------------------------------------------------------------
template <typename TV>
__global__ void k_features(const TV *__restrict__ V0, const int32_t *__restrict__ cols,
                           const int8_t *__restrict__ cls, const double *__restrict__ cent,
                           const double *__restrict__ geom, int ne, double alpha_h,
                           float *__restrict__ feats) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ne) return;
  const double al = geom[24 * ne + l];
  const double diag = (double)V0[(size_t)l * ne + l];
  float *f = feats + (size_t)l * HB_PC_FEATURES;
  int cnt = 0;
  for (int s = 0; s < S; ++s) {
    const int m = cols[l * S + s];
    float *g = f + s * HB_PC_SLOT_FEATURES;
    if (m < 0) {
      for (int q = 0; q < HB_PC_SLOT_FEATURES; ++q) g[q] = 0.0f;
      continue;
    }
    ++cnt;
    const int c = cls[l * S + s];
    const double dx = cent[3 * l] - cent[3 * m], dy = cent[3 * l + 1] - cent[3 * m + 1],
                 dz = cent[3 * l + 2] - cent[3 * m + 2];
    g[0] = (float)((double)V0[(size_t)l * ne + m] / diag);
    g[1] = c == 3 ? 1.0f : 0.0f;
    g[2] = c == 2 ? 1.0f : 0.0f;
    g[3] = c == 1 ? 1.0f : 0.0f;
    g[4] = (float)(sqrt(dx * dx + dy * dy + dz * dz) / sqrt(al));
    g[5] = (float)(geom[24 * ne + m] / al);
    g[6] = (float)(geom[21 * ne + l] * geom[21 * ne + m] + geom[22 * ne + l] * geom[22 * ne + m] +
                   geom[23 * ne + l] * geom[23 * ne + m]);
    g[7] = 1.0f;
  }
  const double hl = sqrt(alpha_h / al);
  f[S * HB_PC_SLOT_FEATURES + 0] = (float)hl;
  f[S * HB_PC_SLOT_FEATURES + 1] = (float)log(hl);
  f[S * HB_PC_SLOT_FEATURES + 2] = (float)cnt / S;
  f[S * HB_PC_SLOT_FEATURES + 3] = 1.0f;
}

// ---------------------------------------------------------------------------------------------
// Normal equations of the sparse approximate inverse of row l: with J = pattern of l and the
// scaled unknowns y = V^0[l,l] m (row l of M is m on J),
//   || m^T V^0[J, :] - e_l^T ||^2 = y^T G y - 2 a^T y + 1,
//   G[s][t] = sum_j V^0[J_s, j] V^0[J_t, j] / V^0[l,l]^2,  a[s] = V^0[J_s, l] / V^0[l,l].
// Absent slots get G = identity, a = 0.  One workgroup per row; rows staged in LDS.  Also
// solves G y = a (the exact minimiser) by Cholesky when y_out is given.
// ---------------------------------------------------------------------------------------------
template <typename TV>
__global__ __launch_bounds__(256) void k_spai_rows(const TV *__restrict__ V0,
                                                   const int32_t *__restrict__ cols, int ne,
                                                   float *__restrict__ gram, float *__restrict__ rhs,
                                                   float *__restrict__ y_out) {
  const int l = blockIdx.x;
  const int tid = threadIdx.x;
  constexpr int CH = 256;
  __shared__ double rows[S][CH];
  __shared__ double G[S][S + 1];
  __shared__ double a[S];
  __shared__ int J[S];
  if (tid < S) J[tid] = cols[l * S + tid];
  __syncthreads();
  // pair (s, t) with s <= t handled by thread tid < 136
  int ps = 0, pt = 0;
  {
    int idx = tid, s = 0;
    while (s < S && idx >= S - s) { idx -= S - s; ++s; }
    ps = s;
    pt = s + idx;
  }
  const bool owner = tid < S * (S + 1) / 2;
  double acc = 0.0;
  for (int j0 = 0; j0 < ne; j0 += CH) {
    for (int e = tid; e < S * CH; e += 256) {
      const int s = e / CH, j = j0 + e % CH;
      const int m = J[s];
      rows[s][e % CH] = (m >= 0 && j < ne) ? (double)V0[(size_t)m * ne + j] : 0.0;
    }
    __syncthreads();
    if (owner)
      for (int j = 0; j < CH; ++j) acc = fma(rows[ps][j], rows[pt][j], acc);
    __syncthreads();
  }
  const double diag = (double)V0[(size_t)l * ne + l];
  const double inv2 = 1.0 / (diag * diag);
  if (owner) {
    double v = acc * inv2;
    if (J[ps] < 0 || J[pt] < 0) v = (ps == pt) ? 1.0 : 0.0;
    G[ps][pt] = v;
    G[pt][ps] = v;
  }
  if (tid < S) a[tid] = J[tid] >= 0 ? (double)V0[(size_t)J[tid] * ne + l] / diag : 0.0;
  __syncthreads();
  if (tid < S * S) gram[(size_t)l * S * S + tid] = (float)G[tid / S][tid % S];
  if (tid < S) rhs[(size_t)l * S + tid] = (float)a[tid];
  if (y_out && tid == 0) {
    // Cholesky of G in place (lower), then two triangular solves
    double Lm[S][S];
    for (int i = 0; i < S; ++i)
      for (int k = 0; k <= i; ++k) {
        double sum = G[i][k];
        for (int q = 0; q < k; ++q) sum -= Lm[i][q] * Lm[k][q];
        Lm[i][k] = (i == k) ? sqrt(fmax(sum, 1e-300)) : sum / Lm[k][k];
      }
    double z[S];
    for (int i = 0; i < S; ++i) {
      double sum = a[i];
      for (int q = 0; q < i; ++q) sum -= Lm[i][q] * z[q];
      z[i] = sum / Lm[i][i];
    }
    for (int i = S - 1; i >= 0; --i) {
      double sum = z[i];
      for (int q = i + 1; q < S; ++q) sum -= Lm[q][i] * z[q];
      z[i] = sum / Lm[i][i];
    }
    for (int i = 0; i < S; ++i) y_out[(size_t)l * S + i] = J[i] >= 0 ? (float)z[i] : 0.0f;
  }
}

// ---------------------------------------------------------------------------------------------
// Dense layers.  Row-major activations X [B][n_in]; weights W [n_out][n_in]; tiles 64 x 64 with
// LDS staging of 16-wide k slices, 4 x 4 outputs per thread.
//   mode 0: Y = X W^T + b          (forward, optional tanh)
//   k_gemm_tn: dW += dY^T X        (weight gradient, [n_out][n_in])
//   k_gemm_nn: dX = dY W           ([B][n_in])
// ---------------------------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void k_dense_fwd(const float *__restrict__ X, const float *__restrict__ W,
                                                   const float *__restrict__ bias, float *__restrict__ Z,
                                                   float *__restrict__ H, int B, int nin, int nout,
                                                   int act) {
  const int b0 = blockIdx.x * GT, o0 = blockIdx.y * GT;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  __shared__ float Xs[GK][GT + 1], Ws[GK][GT + 1];
  float acc[4][4] = {};
  for (int k0 = 0; k0 < nin; k0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e / GK, k = e % GK;
      Xs[k][r] = (b0 + r < B && k0 + k < nin) ? X[(size_t)(b0 + r) * nin + k0 + k] : 0.0f;
      Ws[k][r] = (o0 + r < nout && k0 + k < nin) ? W[(size_t)(o0 + r) * nin + k0 + k] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; ++k) {
      float xa[4], wb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xa[i] = Xs[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) wb[j] = Ws[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(xa[i], wb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = b0 + ty * 4 + i;
    if (b >= B) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = o0 + tx * 4 + j;
      if (o >= nout) continue;
      const float z = acc[i][j] + bias[o];
      Z[(size_t)b * nout + o] = z;
      if (H) H[(size_t)b * nout + o] = act ? tanhf(z) : z;
    }
  }
}

// dW[o][i] = sum_b dY[b][o] X[b][i] over the rows of chunk blockIdx.z (rows per chunk: rpc),
// written to dW + blockIdx.z * nout * nin; grid over (o tiles, i tiles, row chunks)
__global__ __launch_bounds__(256) void k_gemm_tn(const float *__restrict__ dY, const float *__restrict__ X,
                                                 float *__restrict__ dW, int B, int nout, int nin,
                                                 int rpc) {
  const int o0 = blockIdx.x * GT, i0 = blockIdx.y * GT;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  __shared__ float Ds[GK][GT + 1], Xs[GK][GT + 1];
  float acc[4][4] = {};
  const int bb = blockIdx.z * rpc, be = min(B, bb + rpc);
  dW += (size_t)blockIdx.z * nout * nin;
  for (int b0 = bb; b0 < be; b0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e % GT, k = e / GT;
      Ds[k][r] = (b0 + k < be && o0 + r < nout) ? dY[(size_t)(b0 + k) * nout + o0 + r] : 0.0f;
      Xs[k][r] = (b0 + k < be && i0 + r < nin) ? X[(size_t)(b0 + k) * nin + i0 + r] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; ++k) {
      float da[4], xb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) da[i] = Ds[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) xb[j] = Xs[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(da[i], xb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = o0 + ty * 4 + i;
    if (o >= nout) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = i0 + tx * 4 + j;
      if (c < nin) dW[(size_t)o * nin + c] = acc[i][j];
    }
  }
}

// dX[b][i] = sum_o dY[b][o] W[o][i], then (act) dX *= 1 - H^2 (H = tanh of that layer's input)
__global__ __launch_bounds__(256) void k_gemm_nn(const float *__restrict__ dY, const float *__restrict__ W,
                                                 const float *__restrict__ Hin, float *__restrict__ dX,
                                                 int B, int nout, int nin, int act) {
  const int b0 = blockIdx.x * GT, i0 = blockIdx.y * GT;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  __shared__ float Ds[GK][GT + 1], Wsm[GK][GT + 1];
  float acc[4][4] = {};
  for (int k0 = 0; k0 < nout; k0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e / GK, k = e % GK;
      Ds[k][r] = (b0 + r < B && k0 + k < nout) ? dY[(size_t)(b0 + r) * nout + k0 + k] : 0.0f;
    }
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e % GT, k = e / GT;
      Wsm[k][r] = (k0 + k < nout && i0 + r < nin) ? W[(size_t)(k0 + k) * nin + i0 + r] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; ++k) {
      float da[4], wb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) da[i] = Ds[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) wb[j] = Wsm[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(da[i], wb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = b0 + ty * 4 + i;
    if (b >= B) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = i0 + tx * 4 + j;
      if (c >= nin) continue;
      float v = acc[i][j];
      if (act) {
        const float h = Hin[(size_t)b * nin + c];
        v *= 1.0f - h * h;
      }
      dX[(size_t)b * nin + c] = v;
    }
  }
}

// db[o] = sum_b dY[b][o] over the rows of chunk blockIdx.y, written to db + blockIdx.y * n
__global__ void k_colsum(const float *__restrict__ dY, int B, int n, float *__restrict__ db,
                         int rpc) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int bb = blockIdx.y * rpc, be = min(B, bb + rpc);
  float s = 0.0f;
  for (int b = bb; b < be; ++b) s += dY[(size_t)b * n + o];
  db[(size_t)blockIdx.y * n + o] = s;
}

// out[i] = sum_c P[c][i] in a fixed order (deterministic reduction of the row-chunk partials)
__global__ void k_sum_chunks(const float *__restrict__ P, int nc, size_t n, float *__restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float acc = 0.0f;
    for (int c = 0; c < nc; ++c) acc += P[(size_t)c * n + i];
    out[i] = acc;
  }
}

// Row chunks of the weight / bias gradients: enough workgroups to fill the chip, at most
// kMaxChunks partial copies (kept in the backward workspace).
constexpr int kMaxChunks = 32;
inline int grad_chunks(int B) { return std::max(1, std::min(kMaxChunks, (B + 127) / 128)); }

// Quadratic loss per row: L_b = y^T G y - 2 a^T y + 1; dL/dy = 2 (G y - a) / B (mean over rows)
__global__ void k_quadloss(const float *__restrict__ Y, const float *__restrict__ G,
                           const float *__restrict__ a, int B, float *__restrict__ dY,
                           float *__restrict__ rowloss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float *y = Y + (size_t)b * S;
  const float *g = G + (size_t)b * S * S;
  const float *r = a + (size_t)b * S;
  double L = 1.0;
  for (int s = 0; s < S; ++s) {
    double gy = 0.0;
    for (int t = 0; t < S; ++t) gy += (double)g[s * S + t] * y[t];
    L += (double)y[s] * gy - 2.0 * (double)r[s] * y[s];
    if (dY) dY[(size_t)b * S + s] = (float)(2.0 * (gy - r[s]) / B);
  }
  if (rowloss) rowloss[b] = (float)L;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Batch b of the shuffled training rows: Xb[b] = X[idx[i0 + b]] (F floats), Gb, Ab likewise.
// One workgroup per batch row.
__global__ __launch_bounds__(256) void k_gather_rows(const int32_t *__restrict__ idx, int i0,
                                                     const float *__restrict__ X,
                                                     const float *__restrict__ G,
                                                     const float *__restrict__ A, int F,
                                                     float *__restrict__ Xb, float *__restrict__ Gb,
                                                     float *__restrict__ Ab) {
  const int b = blockIdx.x;
  const size_t r = (size_t)idx[i0 + b];
  for (int e = threadIdx.x; e < F; e += blockDim.x) Xb[(size_t)b * F + e] = X[r * F + e];
  for (int e = threadIdx.x; e < S * S; e += blockDim.x) Gb[(size_t)b * S * S + e] = G[r * S * S + e];
  if (threadIdx.x < S) Ab[(size_t)b * S + threadIdx.x] = A[r * S + threadIdx.x];
}

// acc[0] += sum of rl[0 .. B-1] (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_sum_loss(const float *__restrict__ rl, int B,
                                                  double *__restrict__ acc) {
  __shared__ double part[256];
  double v = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) v += (double)rl[b];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += part[0];
}

// M[l][s] = y[l][s] / V^0[l,l] (double)
template <typename TV>
__global__ void k_install(const TV *__restrict__ V0, const float *__restrict__ y, int ne,
                          double *__restrict__ M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne * S) return;
  const int l = i / S;
  M[i] = (double)y[i] / (double)V0[(size_t)l * ne + l];
}

}  // namespace

// z[k][l] = sum_s M[l][s] q[k][cols[l][s]] for every time step k: one lane per slot s (a gather
// each, all in flight together), summed over the HB_PC_SLOTS lanes of (k, l) by a butterfly
static_assert(HB_PC_SLOTS == 16, "the butterfly below sums 16 lanes");
__global__ __launch_bounds__(256) void k_precond_apply(const double *__restrict__ M,
                                                       const int32_t *__restrict__ cols,
                                                       const double *__restrict__ q,
                                                       double *__restrict__ z, int nt, int ne) {
  const size_t n = (size_t)nt * ne;
  const int slot = threadIdx.x & (HB_PC_SLOTS - 1);
  const size_t stride = (size_t)gridDim.x * blockDim.x / HB_PC_SLOTS;
  // the loop bound is the same for the 16 lanes of a group, so each butterfly has all of them
  for (size_t i = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) / HB_PC_SLOTS; i < n; i += stride) {
    const int k = (int)(i / ne), l = (int)(i % ne);
    const int m = cols[l * HB_PC_SLOTS + slot];
    double v = m >= 0 ? M[l * HB_PC_SLOTS + slot] * q[(size_t)k * ne + m] : 0.0;
#pragma unroll
    for (int o = HB_PC_SLOTS / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, HB_PC_SLOTS);
    if (slot == 0) z[i] = v;
  }
}

int precond_apply(hb_ctx *c, const double *q, double *z, hipStream_t s) {
  const size_t n = (size_t)c->nt * c->ne;
  hipLaunchKernelGGL(k_precond_apply, dim3(grid_for(n * HB_PC_SLOTS)), dim3(256), 0, s, c->d_pc_M, c->d_pc_cols,
                     q, z, c->nt, (int)c->ne);
  HB_CHECK_L(c, hipGetLastError());
  return HB_OK;
}

}  // namespace hb

using namespace hb;

namespace {
int lfail(hb_ctx *c, int code, const std::string &m) {
  if (c) c->err = m;
  return code;
}

size_t mlp_nparams(const hb_mlp_dims *d) {
  return (size_t)d->n_hidden * d->n_in + d->n_hidden + (size_t)d->n_hidden * d->n_hidden +
         d->n_hidden + (size_t)d->n_out * d->n_hidden + d->n_out;
}

bool dims_ok(const hb_mlp_dims *d) {
  return d && d->n_in > 0 && d->n_hidden > 0 && d->n_out > 0 && d->n_in <= 4096 &&
         d->n_hidden <= 4096 && d->n_out <= 4096;
}

int gfail(int code, const std::string &m) {
  hb::set_global_error(m);
  return code;
}

// splitmix64 (Steele, Lea, Flood 2014): the seeded sequence of initial weights and row orders
uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t &x) { return (double)(splitmix64(x) >> 11) * (1.0 / 9007199254740992.0); }

// device buffers released on every return path
struct DevFloats {
  float *p = nullptr;
  ~DevFloats() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

struct hb_pcnet {
  hb_mlp_dims dims{};
  float *d_params = nullptr;
  size_t n = 0;
};

namespace {
bool pc_dims(const hb_mlp_dims *d) {
  return dims_ok(d) && d->n_in == HB_PC_FEATURES && d->n_out == HB_PC_SLOTS;
}

int new_net(const hb_mlp_dims &d, const float *host_params, hb_pcnet **out) {
  hb_pcnet *net = new hb_pcnet;
  net->dims = d;
  net->n = mlp_nparams(&d);
  if (hipMalloc(&net->d_params, sizeof(float) * net->n) != hipSuccess) {
    delete net;
    return gfail(HB_ENOMEM, "hipMalloc of the network parameters failed");
  }
  if (host_params &&
      hipMemcpy(net->d_params, host_params, sizeof(float) * net->n, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(net->d_params);
    delete net;
    return gfail(HB_EHIP, "copy of the network parameters failed");
  }
  *out = net;
  return HB_OK;
}
}  // namespace

extern "C" {

int64_t hb_mlp_num_params(const hb_mlp_dims *d) { return dims_ok(d) ? (int64_t)mlp_nparams(d) : -1; }

int64_t hb_mlp_work_floats(const hb_mlp_dims *d, int64_t batch) {
  if (!dims_ok(d) || batch <= 0) return -1;
  const int64_t H = d->n_hidden, wmax = H * std::max<int64_t>(std::max<int64_t>(H, d->n_in), d->n_out);
  return batch * (4 * H + d->n_out) + batch * 2 * H + (int64_t)kMaxChunks * (wmax + H);
}

int hb_precond_pattern(hb_ctx *c, int32_t *cols, int8_t *cls, void *stream) {
  if (!c || !cols) return lfail(c, HB_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  HB_CHECK_L(c, hipMemcpyAsync(cols, c->d_pc_cols, sizeof(int32_t) * c->ne * HB_PC_SLOTS,
                               hipMemcpyDeviceToDevice, s));
  if (cls)
    HB_CHECK_L(c, hipMemcpyAsync(cls, c->d_pc_cls, c->ne * HB_PC_SLOTS, hipMemcpyDeviceToDevice, s));
  return HB_OK;
}

int hb_precond_features(hb_ctx *c, float *feats, void *stream) {
  if (!c || !feats) return lfail(c, HB_EINVAL, "null argument");
  if (c->nu) return lfail(c, HB_EINVAL, "not available on a non-uniform time grid");
  if (!c->have_V) return lfail(c, HB_ESTATE, "V not assembled");
  hipStream_t s = (hipStream_t)stream;
  const int ne = (int)c->ne;
  if (c->storage_f32)
    hipLaunchKernelGGL(k_features<float>, dim3((ne + 255) / 256), dim3(256), 0, s, (const float *)c->d_V,
                       c->d_pc_cols, c->d_pc_cls, c->d_cent, c->d_geom, ne, c->alpha * c->h, feats);
  else
    hipLaunchKernelGGL(k_features<double>, dim3((ne + 255) / 256), dim3(256), 0, s, (const double *)c->d_V,
                       c->d_pc_cols, c->d_pc_cls, c->d_cent, c->d_geom, ne, c->alpha * c->h, feats);
  HB_CHECK_L(c, hipGetLastError());
  return HB_OK;
}

int hb_precond_spai(hb_ctx *c, float *gram, float *rhs, float *weights, void *stream) {
  if (!c || !gram || !rhs) return lfail(c, HB_EINVAL, "null argument");
  if (c->nu) return lfail(c, HB_EINVAL, "not available on a non-uniform time grid");
  if (!c->have_V) return lfail(c, HB_ESTATE, "V not assembled");
  hipStream_t s = (hipStream_t)stream;
  const int ne = (int)c->ne;
  if (c->storage_f32)
    hipLaunchKernelGGL(k_spai_rows<float>, dim3(ne), dim3(256), 0, s, (const float *)c->d_V, c->d_pc_cols,
                       ne, gram, rhs, weights);
  else
    hipLaunchKernelGGL(k_spai_rows<double>, dim3(ne), dim3(256), 0, s, (const double *)c->d_V, c->d_pc_cols,
                       ne, gram, rhs, weights);
  HB_CHECK_L(c, hipGetLastError());
  return HB_OK;
}

int hb_precond_set(hb_ctx *c, const float *weights, void *stream) {
  if (!c) return lfail(c, HB_EINVAL, "null context");
  if (c->nu) return lfail(c, HB_EINVAL, "not available on a non-uniform time grid");
  if (!weights) {
    c->pc_active = false;
    return HB_OK;
  }
  if (!c->have_V) return lfail(c, HB_ESTATE, "V not assembled");
  hipStream_t s = (hipStream_t)stream;
  const int ne = (int)c->ne;
  if (!c->d_pc_M) HB_CHECK_L(c, hipMalloc(&c->d_pc_M, sizeof(double) * ne * HB_PC_SLOTS));
  const int n = ne * HB_PC_SLOTS;
  if (c->storage_f32)
    hipLaunchKernelGGL(k_install<float>, dim3((n + 255) / 256), dim3(256), 0, s, (const float *)c->d_V,
                       weights, ne, c->d_pc_M);
  else
    hipLaunchKernelGGL(k_install<double>, dim3((n + 255) / 256), dim3(256), 0, s, (const double *)c->d_V,
                       weights, ne, c->d_pc_M);
  HB_CHECK_L(c, hipGetLastError());
  c->pc_active = true;
  return HB_OK;
}

int hb_mlp_forward(const hb_mlp_dims *d, const float *params, const float *x, int64_t batch,
                   float *y, float *work, void *stream) {
  if (!dims_ok(d) || !params || !x || !y || !work || batch <= 0 || batch > (1 << 26)) return HB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)batch, I = d->n_in, H = d->n_hidden, O = d->n_out;
  const float *W1 = params, *b1 = W1 + (size_t)H * I, *W2 = b1 + H, *b2 = W2 + (size_t)H * H;
  const float *W3 = b2 + H, *b3 = W3 + (size_t)O * H;
  float *Z1 = work, *H1 = Z1 + (size_t)B * H, *Z2 = H1 + (size_t)B * H, *H2 = Z2 + (size_t)B * H;
  float *Z3 = H2 + (size_t)B * H;
  dim3 g1((B + GT - 1) / GT, (H + GT - 1) / GT), g3((B + GT - 1) / GT, (O + GT - 1) / GT);
  hipLaunchKernelGGL(k_dense_fwd, g1, dim3(256), 0, s, x, W1, b1, Z1, H1, B, I, H, 1);
  hipLaunchKernelGGL(k_dense_fwd, g1, dim3(256), 0, s, H1, W2, b2, Z2, H2, B, H, H, 1);
  hipLaunchKernelGGL(k_dense_fwd, g3, dim3(256), 0, s, H2, W3, b3, Z3, y, B, H, O, 0);
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

int hb_mlp_backward(const hb_mlp_dims *d, const float *params, const float *x, int64_t batch,
                    const float *work, const float *dy, float *grads, void *stream) {
  if (!dims_ok(d) || !params || !x || !dy || !grads || !work || batch <= 0 || batch > (1 << 26))
    return HB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)batch, I = d->n_in, H = d->n_hidden, O = d->n_out;
  const float *W2 = params + (size_t)H * I + H, *W3 = W2 + (size_t)H * H + H;
  const float *H1 = work + (size_t)B * H, *H2 = work + (size_t)3 * B * H;
  float *dW1 = grads, *db1 = dW1 + (size_t)H * I, *dW2 = db1 + H, *db2 = dW2 + (size_t)H * H;
  float *dW3 = db2 + H, *db3 = dW3 + (size_t)O * H;
  float *dZ2 = (float *)work + (size_t)B * (4 * H + O), *dZ1 = dZ2 + (size_t)B * H;
  // row-chunk partials of the weight and bias gradients, then a fixed-order sum
  const int nc = grad_chunks(B), rpc = (B + nc - 1) / nc;
  const int64_t wmax = (int64_t)H * std::max(std::max(H, I), O);
  float *Pw = dZ1 + (size_t)B * H, *Pb = Pw + (size_t)kMaxChunks * wmax;
  auto weight_grad = [&](const float *dY, const float *X, float *dW, int nout, int nin) {
    hipLaunchKernelGGL(k_gemm_tn, dim3((nout + GT - 1) / GT, (nin + GT - 1) / GT, nc), dim3(256), 0, s,
                       dY, X, Pw, B, nout, nin, rpc);
    const size_t n = (size_t)nout * nin;
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for(n)), dim3(256), 0, s, Pw, nc, n, dW);
  };
  auto bias_grad = [&](const float *dY, float *db, int n) {
    hipLaunchKernelGGL(k_colsum, dim3((n + 255) / 256, nc), dim3(256), 0, s, dY, B, n, Pb, rpc);
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_for((size_t)n)), dim3(256), 0, s, Pb, nc, (size_t)n, db);
  };
  // layer 3 (linear): dW3 = dy^T H2, db3 = sum dy, dZ2 = (dy W3) * (1 - H2^2)
  weight_grad(dy, H2, dW3, O, H);
  bias_grad(dy, db3, O);
  hipLaunchKernelGGL(k_gemm_nn, dim3((B + GT - 1) / GT, (H + GT - 1) / GT), dim3(256), 0, s, dy, W3, H2, dZ2, B, O, H, 1);
  // layer 2
  weight_grad(dZ2, H1, dW2, H, H);
  bias_grad(dZ2, db2, H);
  hipLaunchKernelGGL(k_gemm_nn, dim3((B + GT - 1) / GT, (H + GT - 1) / GT), dim3(256), 0, s, dZ2, W2, H1, dZ1, B, H, H, 1);
  // layer 1
  weight_grad(dZ1, x, dW1, H, I);
  bias_grad(dZ1, db1, H);
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

int hb_precond_loss(const float *y, const float *gram, const float *rhs, int64_t rows, float *dy,
                    float *rowloss, void *stream) {
  if (!y || !gram || !rhs || rows <= 0 || rows > (1 << 26)) return HB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_quadloss, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, y, gram, rhs,
                     (int)rows, dy, rowloss);
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

void hb_default_train_opts(hb_train_opts *o) {
  if (!o) return;
  *o = hb_train_opts{};
  o->epochs = 30;
  o->batch = 2048;
  o->lr = 1e-3f;
  o->n_hidden = 256;
  o->seed = 0;
}

int hb_pcnet_create(const hb_mlp_dims *dims, const float *params, hb_pcnet **out) {
  if (!out || !params) return gfail(HB_EINVAL, "null argument");
  if (!pc_dims(dims)) return gfail(HB_EINVAL, "dims must be (HB_PC_FEATURES, 1..4096, HB_PC_SLOTS)");
  return new_net(*dims, params, out);
}

int hb_pcnet_get(const hb_pcnet *net, hb_mlp_dims *dims, float *params) {
  if (!net) return gfail(HB_EINVAL, "null network");
  if (dims) *dims = net->dims;
  if (params && hipMemcpy(params, net->d_params, sizeof(float) * net->n, hipMemcpyDeviceToHost) != hipSuccess)
    return gfail(HB_EHIP, "copy of the network parameters failed");
  return HB_OK;
}

void hb_pcnet_destroy(hb_pcnet *net) {
  if (!net) return;
  if (net->d_params) (void)hipFree(net->d_params);
  delete net;
}

int hb_pcnet_save(const hb_pcnet *net, const char *path) {
  if (!net || !path) return gfail(HB_EINVAL, "null argument");
  std::vector<float> p(net->n);
  int rc = hb_pcnet_get(net, nullptr, p.data());
  if (rc) return rc;
  FILE *f = fopen(path, "wb");
  if (!f) return gfail(HB_EINVAL, std::string("cannot open ") + path + " for writing");
  const int32_t d[3] = {net->dims.n_in, net->dims.n_hidden, net->dims.n_out};
  const int64_t n = (int64_t)net->n;
  bool ok = fwrite("HBPCNET1", 1, 8, f) == 8 && fwrite(d, sizeof(int32_t), 3, f) == 3 &&
            fwrite(&n, sizeof(int64_t), 1, f) == 1 && fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? HB_OK : gfail(HB_EINVAL, std::string("write to ") + path + " failed");
}

int hb_pcnet_load(const char *path, hb_pcnet **out) {
  if (!path || !out) return gfail(HB_EINVAL, "null argument");
  FILE *f = fopen(path, "rb");
  if (!f) return gfail(HB_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  int32_t d[3];
  int64_t n = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "HBPCNET1", 8) == 0 &&
            fread(d, sizeof(int32_t), 3, f) == 3 && fread(&n, sizeof(int64_t), 1, f) == 1;
  hb_mlp_dims dims{d[0], d[1], d[2]};
  ok = ok && pc_dims(&dims) && n == (int64_t)mlp_nparams(&dims);
  std::vector<float> p;
  if (ok) {
    p.resize((size_t)n);
    ok = fread(p.data(), sizeof(float), p.size(), f) == p.size() && fgetc(f) == EOF;
  }
  fclose(f);
  if (!ok) return gfail(HB_EINVAL, std::string(path) + " is not a complete network file of this library");
  return new_net(dims, p.data(), out);
}

int hb_precond_install(hb_ctx *c, const hb_pcnet *net, void *stream) {
  if (!c) return gfail(HB_EINVAL, "null context");
  if (!net) return lfail(c, HB_EINVAL, "null network");
  if (!c->have_V) return lfail(c, HB_ESTATE, "V not assembled");
  hipStream_t s = (hipStream_t)stream;
  const int64_t ne = c->ne;
  const int64_t nw = hb_mlp_work_floats(&net->dims, ne);
  const size_t need = (size_t)ne * (HB_PC_FEATURES + HB_PC_SLOTS) + (size_t)nw;
  if (c->pc_buf_n < need) {
    if (c->d_pc_buf) (void)hipFree(c->d_pc_buf);
    c->d_pc_buf = nullptr;
    c->pc_buf_n = 0;
    HB_CHECK_L(c, hipMalloc(&c->d_pc_buf, sizeof(float) * need));
    c->pc_buf_n = need;
  }
  float *feats = c->d_pc_buf, *y = feats + (size_t)ne * HB_PC_FEATURES, *work = y + (size_t)ne * HB_PC_SLOTS;
  int rc = hb_precond_features(c, feats, stream);
  if (rc) return rc;
  if ((rc = hb_mlp_forward(&net->dims, net->d_params, feats, ne, y, work, stream)))
    return lfail(c, rc, "MLP forward pass failed");
  return hb_precond_set(c, y, s);
}

int hb_precond_train(hb_ctx *const *ctxs, int32_t n_ctx, const hb_train_opts *opts, hb_pcnet **out,
                     float *epoch_loss, void *stream) {
  if (!ctxs || n_ctx < 1 || !out) return gfail(HB_EINVAL, "need at least one context and an output");
  hb_ctx *c0 = ctxs[0];
  if (!c0) return gfail(HB_EINVAL, "null context");
  hb_train_opts o;
  hb_default_train_opts(&o);
  if (opts) {
    for (int i = 0; i < 8; ++i)
      if (opts->reserved[i]) return lfail(c0, HB_EINVAL, "hb_train_opts.reserved must be zero");
    if (opts->epochs > 0) o.epochs = opts->epochs;
    if (opts->batch > 0) o.batch = opts->batch;
    if (opts->lr > 0) o.lr = opts->lr;
    if (opts->n_hidden > 0) o.n_hidden = opts->n_hidden;
    o.seed = opts->seed;
  }
  if (o.n_hidden > 4096 || o.epochs > 100000) return lfail(c0, HB_EINVAL, "n_hidden <= 4096, epochs <= 100000");
  int64_t R = 0;
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) return lfail(c0, HB_EINVAL, "null context in the list");
    if (ctxs[i]->nu) return lfail(c0, HB_EINVAL, "training contexts need a uniform time grid");
    if (!ctxs[i]->have_V) return lfail(c0, HB_ESTATE, "V not assembled on a training context");
    R += ctxs[i]->ne;
  }
  if (R > (1 << 26)) return lfail(c0, HB_EINVAL, "too many training rows");
  hipStream_t s = (hipStream_t)stream;
  constexpr int F = HB_PC_FEATURES;
  const hb_mlp_dims dims{F, o.n_hidden, S};
  const int B = (int)std::min<int64_t>(o.batch, R);
  const size_t np = mlp_nparams(&dims);
  const int64_t nw = hb_mlp_work_floats(&dims, B);
  // training rows: features, Gram matrices, right-hand sides of every context
  DevFloats data, batch, state;
  HB_CHECK_L(c0, hipMalloc(&data.p, sizeof(float) * (size_t)R * (F + S * S + S)));
  float *X = data.p, *G = X + (size_t)R * F, *A = G + (size_t)R * S * S;
  int64_t off = 0;
  for (int i = 0; i < n_ctx; ++i) {
    hb_ctx *c = ctxs[i];
    int rc = hb_precond_features(c, X + off * F, stream);
    if (!rc) rc = hb_precond_spai(c, G + off * S * S, A + off * S, nullptr, stream);
    if (rc) return lfail(c0, rc, c->err);
    off += c->ne;
  }
  // batch buffers: Xb, Gb, Ab, y, dy, rowloss, MLP workspace, shuffled row indices, loss sum
  const size_t nb = (size_t)B * (F + S * S + S + S + S + 1) + (size_t)nw + (size_t)R + 4;
  HB_CHECK_L(c0, hipMalloc(&batch.p, sizeof(float) * nb));
  float *Xb = batch.p, *Gb = Xb + (size_t)B * F, *Ab = Gb + (size_t)B * S * S, *y = Ab + (size_t)B * S;
  float *dy = y + (size_t)B * S, *rl = dy + (size_t)B * S, *work = rl + B;
  int32_t *idx = (int32_t *)(work + nw);
  double *acc = (double *)(((uintptr_t)(idx + R) + 7) & ~(uintptr_t)7);
  // parameters, gradients and Adam moments; Glorot-uniform weights, zero biases
  std::vector<float> p0(np, 0.0f);
  {
    uint64_t st = o.seed;
    size_t q = 0;
    const int fan[3][2] = {{F, o.n_hidden}, {o.n_hidden, o.n_hidden}, {o.n_hidden, S}};
    for (int L = 0; L < 3; ++L) {
      const double lim = std::sqrt(6.0 / (fan[L][0] + fan[L][1]));
      for (size_t e = 0; e < (size_t)fan[L][0] * fan[L][1]; ++e)
        p0[q++] = (float)((2.0 * uniform01(st) - 1.0) * lim);
      q += fan[L][1];  // biases stay zero
    }
  }
  hb_pcnet *net = nullptr;
  int rc = new_net(dims, p0.data(), &net);
  if (rc) return lfail(c0, rc, "network allocation failed");
  std::unique_ptr<hb_pcnet, void (*)(hb_pcnet *)> owner(net, hb_pcnet_destroy);
  HB_CHECK_L(c0, hipMalloc(&state.p, sizeof(float) * 3 * np));
  float *grads = state.p, *m1 = grads + np, *m2 = m1 + np;
  HB_CHECK_L(c0, hipMemsetAsync(m1, 0, sizeof(float) * 2 * np, s));
  std::vector<int32_t> perm((size_t)R);
  uint64_t st = o.seed ^ 0x5DEECE66DULL;
  int step = 0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    for (int64_t i = 0; i < R; ++i) perm[(size_t)i] = (int32_t)i;
    for (int64_t i = R - 1; i > 0; --i) {  // Fisher-Yates
      const int64_t j = (int64_t)(splitmix64(st) % (uint64_t)(i + 1));
      std::swap(perm[(size_t)i], perm[(size_t)j]);
    }
    HB_CHECK_L(c0, hipMemcpyAsync(idx, perm.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice, s));
    HB_CHECK_L(c0, hipMemsetAsync(acc, 0, sizeof(double), s));
    int nbatch = 0;
    for (int64_t i0 = 0; i0 + B <= R; i0 += B, ++nbatch) {
      hipLaunchKernelGGL(k_gather_rows, dim3(B), dim3(256), 0, s, idx, (int)i0, X, G, A, F, Xb, Gb, Ab);
      if ((rc = hb_mlp_forward(&dims, net->d_params, Xb, B, y, work, stream)) ||
          (rc = hb_precond_loss(y, Gb, Ab, B, dy, rl, stream)) ||
          (rc = hb_mlp_backward(&dims, net->d_params, Xb, B, work, dy, grads, stream)) ||
          (rc = hb_adam_step(net->d_params, grads, m1, m2, (int64_t)np, o.lr, 0.9f, 0.999f, 1e-8f,
                             ++step, stream)))
        return lfail(c0, rc, "training step failed");
      hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, rl, B, acc);
    }
    double tot = 0.0;
    HB_CHECK_L(c0, hipMemcpyAsync(&tot, acc, sizeof(double), hipMemcpyDeviceToHost, s));
    HB_CHECK_L(c0, hipStreamSynchronize(s));  // also keeps perm alive until its copy is done
    if (epoch_loss) epoch_loss[ep] = (float)(tot / std::max(1, nbatch * B));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lfail(c0, HB_EHIP, std::string("training: ") + hipGetErrorString(e));
  *out = owner.release();
  return HB_OK;
}

int hb_adam_step(float *params, const float *grads, float *m, float *v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (!params || !grads || !m || !v || n <= 0 || step < 1) return HB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for((size_t)n)), dim3(256), 0, s, params, grads, m, v, (size_t)n, lr,
                     beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? HB_OK : HB_EHIP;
}

}  // extern "C"
