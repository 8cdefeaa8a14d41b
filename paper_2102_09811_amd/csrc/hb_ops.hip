// Operations on assembled blocks: block-Toeplitz apply (Sec. 3.1 eq. for V_h w, Sec. 3.2 eq. for
// K_h), the Dirichlet right-hand side (Sec. 3.4), solvers for V_h w = b, and the representation
// formula (potentials of Sec. 3.5).  All vectors are time-major: entry [k * n + j].
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hb_device.h"
#include "hb_internal.h"

namespace hb {
namespace {

#define HB_CHECK(ctx, call)                                                               \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                     \
      return e_ == hipErrorOutOfMemory ? HB_ENOMEM : HB_EHIP;                             \
    }                                                                                     \
  } while (0)

// ------------------------------------------------------------------------------------------
// Block-Toeplitz product Y[k][r] = sum_{d <= k} sum_c A^d[r][c] X[k-d][c] on MFMA
// (v_mfma_f64_16x16x4 for double blocks, v_mfma_f32_16x16x4 for float blocks).
// Workgroup = 64 rows (wave w: rows 16w..16w+15) x all E_t time steps, for the column chunks of
// its group g and the blocks d = dlo + z, dlo + z + slices, ... of its slice z.  Per 32-column
// chunk the source X[:, chunk] is staged in LDS once, behind 16 zero rows, and serves every d
// (the time shift k - d is applied when reading it).  A streams from HBM straight into MFMA
// fragments: lane l (lm = l % 16, lk = l / 16) loads the 8 consecutive entries
// A^d[row 16w + lm][c0 + 8 lk .. + 8] and feeds entry s as the k = lk operand of step s, matched
// by the B operand X[time 16n + lm - d][c0 + 8 lk + s] (the steps cover the 32 columns in a
// permuted order).  The next d's fragment is loaded while the current one runs.  Time chunks
// that end before d are skipped.  Each (g, z) writes the partial result P[g][z][k][r];
// k_sum_groups adds them in a fixed order.
// ------------------------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int TR = 64;   // rows per workgroup
constexpr int kTC = 32;  // columns per chunk
constexpr int kXS = kTC + 1;
constexpr int kFE = kTC / 4;  // fragment entries per lane (consecutive columns of one row)
static_assert(kBlockPad >= (kTC - 1) * sizeof(double), "fragment loads past the last row");

template <typename TA> struct Mfma;
template <> struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register i of lane (lm, lk) holds row lk + 4 i, column lm
  static __device__ __forceinline__ int row(int lk, int i) { return lk + 4 * i; }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register i of lane (lm, lk) holds row 4 lk + i, column lm
  static __device__ __forceinline__ int row(int lk, int i) { return 4 * lk + i; }
};

// This lane's kFE consecutive entries of a block row.  No bounds test: rows past the block are
// clamped by the caller (their outputs are never stored), entries past the row end belong to the
// next row or to the zeroed tail of the storage (hb_internal.h: kBlockPad) and meet zeros of the
// staged X, so every fragment is kFE / 4 (float) or kFE / 2 (double) plain 16-byte loads.
template <typename TA>
__device__ __forceinline__ void load_frag(TA (&a)[kFE], const TA *__restrict__ p) {
  __builtin_memcpy(a, p, kFE * sizeof(TA));
}

// MFMA steps of block d with fragment a for the time chunks NS..NTC-1 (sources outside the
// requested time window are staged as zeros, so no chunk needs a runtime skip: a data-dependent
// branch here costs the accumulators their registers).
template <typename TA, int NTC, int NS>
__device__ __forceinline__ void toeplitz_block(typename Mfma<TA>::acc_t (&acc)[NTC], const TA (&a)[kFE],
                                               const TA *Xs, int d, int lm, int lk) {
#pragma unroll
  for (int n = NS; n < NTC; ++n) {
    const TA *xb = Xs + (16 + 16 * n + lm - d) * kXS + kFE * lk;
#pragma unroll
    for (int s = 0; s < kFE; ++s) acc[n] = Mfma<TA>::mma(a[s], xb[s], acc[n]);
  }
}

// The blocks d0, d0 + ds, d0 + 2 ds, ... below d1 whose nonzero output times all lie in the time
// chunks NS..NTC-1.  On entry a holds the fragment of the first such block at or after 16 NS (if
// there is one); two fragment buffers alternate, the next block's loads in flight while a block
// is multiplied.
template <typename TA, int NTC, int NS>
struct ToeplitzRange {
  typedef typename Mfma<TA>::acc_t acc_t;
  static __device__ __forceinline__ void run(acc_t (&acc)[NTC], TA (&a)[kFE], const TA *Xs,
                                             const TA *arow, size_t blk, int d0, int d1, int ds,
                                             int lm, int lk) {
    if constexpr (NS < NTC) {
      const int lo = max(d0, 16 * NS), dhi = min(d1, 16 * NS + 16);
      int d = d0 + (lo - d0 + ds - 1) / ds * ds;
      for (; d + ds < dhi; d += 2 * ds) {
        TA b[kFE];
        load_frag(b, arow + (size_t)(d + ds) * blk);
        toeplitz_block<TA, NTC, NS>(acc, a, Xs, d, lm, lk);
        if (d + 2 * ds < d1) load_frag(a, arow + (size_t)(d + 2 * ds) * blk);
        toeplitz_block<TA, NTC, NS>(acc, b, Xs, d + ds, lm, lk);
      }
      if (d < dhi) {
        TA b[kFE];
        if (d + ds < d1) load_frag(b, arow + (size_t)(d + ds) * blk);
        toeplitz_block<TA, NTC, NS>(acc, a, Xs, d, lm, lk);
        if (d + ds < d1) {
#pragma unroll
          for (int s = 0; s < kFE; ++s) a[s] = b[s];
        }
      }
      ToeplitzRange<TA, NTC, NS + 1>::run(acc, a, Xs, arow, blk, d0, d1, ds, lm, lk);
    }
  }
};

template <typename TA, int NTC>
__global__ __launch_bounds__(256) void k_toeplitz(const TA *__restrict__ A,
                                                  const double *__restrict__ X,
                                                  TA *__restrict__ P, int nt, int R, int C,
                                                  int cpg, int dlo, int dhi, int jlo, int jhi,
                                                  int klo, int khi) {
  typedef Mfma<TA> M;
  constexpr int NT = 16 * NTC;
  __shared__ TA Xs[(NT + 16) * kXS];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lm = lane & 15, lk = lane >> 4;
  const int r = blockIdx.x * TR + 16 * w + lm;  // A row of this lane's fragments
  const int g = blockIdx.y, z = blockIdx.z;
  const int nchunk = (C + kTC - 1) / kTC;
  const int q0 = g * cpg, q1 = min(q0 + cpg, nchunk);
  const int d0 = dlo + z, d1 = dhi, ds = gridDim.z;  // interleaved: equal work per slice
  typename M::acc_t acc[NTC];
#pragma unroll
  for (int n = 0; n < NTC; ++n) acc[n] = M::zero();
  const size_t blk = (size_t)R * C;
  for (int q = q0; q < q1 && d0 < d1; ++q) {
    const int c0 = q * kTC;
    __syncthreads();  // the previous chunk is no longer read
    for (int e = tid; e < (NT + 16) * kTC; e += 256) {
      const int row = e / kTC, col = e % kTC, j = row - 16, c = c0 + col;
      Xs[row * kXS + col] = (j >= jlo && j < jhi && c < C) ? (TA)X[(size_t)j * C + c] : TA(0);
    }
    __syncthreads();
    const TA *arow = A + (size_t)min(r, R - 1) * C + c0 + kFE * lk;
    TA a[kFE];
    load_frag(a, arow + (size_t)d0 * blk);
    ToeplitzRange<TA, NTC, 0>::run(acc, a, Xs, arow, blk, d0, d1, ds, lm, lk);
  }
  const int part = g * gridDim.z + z;
#pragma unroll
  for (int n = 0; n < NTC; ++n) {
    const int k = 16 * n + lm;
    if (k < klo || k >= khi) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = blockIdx.x * TR + 16 * w + M::row(lk, i);
      if (rr < R) P[((size_t)part * nt + k) * R + rr] = acc[n][i];
    }
  }
}

// Y[i] = sum_g P[g][i] for i in [i0, i1) (sub: Y[i] -= that sum), added in double in a fixed
// order; n is the stride between the parts
template <typename TP>
__global__ void k_sum_groups(const TP *__restrict__ P, int G, size_t n, double *__restrict__ Y,
                             int sub, size_t i0, size_t i1) {
  for (size_t i = i0 + blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < i1; i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    int g = 0;
    for (; g + 8 <= G; g += 8) {  // eight loads in flight, added in order
      TP v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = P[(size_t)(g + u) * n + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; g < G; ++g) s += (double)P[(size_t)g * n + i];
    if (!sub) Y[i] = s;
    else Y[i] -= s;
  }
}

__global__ void k_to_float(const double *__restrict__ x, float *__restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

__global__ void k_fill(double *__restrict__ y, size_t n, double v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = v;
}

// y_{row} = sum_c A[row][c] x[c], one wave per row; batched over nd matrices A + d * stride
// writing out[(k_out0 + d) * R + row] = beta * out + alpha * y.  A lane reads kGemvBatch columns
// 64 apart per round, all loads issued before the products, so a row of up to 64 kGemvBatch
// columns costs one memory latency rather than one per group of columns.
constexpr int kGemvBatch = 20;

template <typename TA>
__global__ __launch_bounds__(256) void k_gemv_rows(const TA *__restrict__ A, size_t stride,
                                                   const double *__restrict__ x, double *out,
                                                   int R, int C, double alpha, double beta,
                                                   size_t out_stride) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int d = blockIdx.y;
  if (row >= R) return;
  const TA *a = A + (size_t)d * stride + (size_t)row * C;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < C; c0 += 64 * kGemvBatch) {
    TA av[kGemvBatch];
    double xv[kGemvBatch];
#pragma unroll
    for (int u = 0; u < kGemvBatch; ++u) {
      const int c = c0 + lane + 64 * u;
      av[u] = c < C ? a[c] : TA(0);
      xv[u] = c < C ? x[c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kGemvBatch; ++u) s[u & 3] = fma((double)av[u], xv[u], s[u & 3]);
  }
  double t = (s[0] + s[1]) + (s[2] + s[3]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (lane == 0) {
    double *o = out + (size_t)d * out_stride + row;
    *o = beta == 0.0 ? alpha * t : beta * (*o) + alpha * t;  // beta = 0: out is not read
  }
}

// b[k][l] += (h/2) sum_{j in panel l} (area_l / 3) g[k][j]   (the 1/2 M_h g part)
__global__ void k_mass_half(const double *__restrict__ mass, const int32_t *__restrict__ tris,
                            const double *__restrict__ g, double *__restrict__ b, int nt, int ne,
                            int nv, double half_h) {
  const size_t n = (size_t)nt * ne;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / ne), l = (int)(i % ne);
    const double *gk = g + (size_t)k * nv;
    b[i] += half_h * (mass[3 * l] * gk[tris[3 * l]] + mass[3 * l + 1] * gk[tris[3 * l + 1]] +
                      mass[3 * l + 2] * gk[tris[3 * l + 2]]);
  }
}

// The same with step lengths h_k of a non-uniform grid: b[k][l] += h_k / 2 (M_x g^k)_l.
__global__ void k_mass_half_steps(const double *__restrict__ mass, const int32_t *__restrict__ tris,
                                  const double *__restrict__ g, double *__restrict__ b, int nt,
                                  int ne, int nv, const double *__restrict__ hk) {
  const size_t n = (size_t)nt * ne;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / ne), l = (int)(i % ne);
    const double *gk = g + (size_t)k * nv;
    b[i] += 0.5 * hk[k] * (mass[3 * l] * gk[tris[3 * l]] + mass[3 * l + 1] * gk[tris[3 * l + 1]] +
                           mass[3 * l + 2] * gk[tris[3 * l + 2]]);
  }
}

// Neumann right-hand side: on entry b = K_h^T psi; b[k][i] <- half_h sum over the panels l at
// vertex i of (area_l / 3) psi[k][l] - b[k][i], i.e. b = 1/2 M_h^T psi - K_h^T psi.
__global__ void k_mass_half_T(const double *__restrict__ mass, const int32_t *__restrict__ vstart,
                              const int32_t *__restrict__ vadj, const double *__restrict__ psi,
                              double *__restrict__ b, int nt, int ne, int nv, double half_h) {
  const size_t n = (size_t)nt * nv;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / nv), v = (int)(i % nv);
    const double *pk = psi + (size_t)k * ne;
    double acc = 0.0;
    for (int e = vstart[v]; e < vstart[v + 1]; ++e) acc = fma(mass[3 * vadj[2 * e] + vadj[2 * e + 1]], pk[vadj[2 * e]], acc);
    b[i] = half_h * acc - b[i];
  }
}

// ---- inverse by blocked Gauss-Jordan elimination (no pivoting), one launch per panel ----
// Panel R = C = [p0, p0 + b) (b <= kGJB), out of place X -> Y, with P^{-1} = X[R, C]^{-1}:
//   Y[R, :] = P^{-1} X[R, :]                        (the pivot columns: P^{-1}),
//   Y[i, :] = X[i, :] - X[i, C] P^{-1} X[R, :]      for i outside R (the pivot columns:
//                                                   -X[i, C] P^{-1}),
// which is b steps of scalar Gauss-Jordan at once.  Every workgroup (a 64 x 64 tile of Y) inverts
// the pivot block itself -- wave 0, one row per lane in registers, the pivot row broadcast with
// readlane, while the other waves stage X[R, tile columns] and X[tile rows, C] -- then forms its
// slice of T = P^{-1} X[R, tile columns] and updates the tile with a rank-b product, both on MFMA.
constexpr int kGJB = 32;

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(256) void k_gj_step(const double *__restrict__ X,
                                                 double *__restrict__ Y, int n, int p0, int b,
                                                 size_t zs) {
  // blockIdx.z: the matrix of a batch, zs doubles apart
  X += blockIdx.z * zs;
  Y += blockIdx.z * zs;
  __shared__ double Pi[kGJB][kGJB + 1];
  __shared__ double Rr[kGJB][64 + 1];
  __shared__ double Cs[64][kGJB + 1];
  __shared__ double Ts[kGJB][64 + 1];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lm = lane & 15, lk = lane >> 4;
  // this lane's 16 entries of the tile, loaded now so that their latency hides behind the rest
  double xt[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = c0 + 16 * q + lm;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = r0 + 16 * w + lk + 4 * i;
      xt[q][i] = (row < n && col < n) ? X[(size_t)row * n + col] : 0.0;
    }
  }
  if (w == 0) {
    // P padded with the identity to kGJB x kGJB; lane i holds row i (lanes >= kGJB: zeros)
    double row[kGJB];
#pragma unroll
    for (int j = 0; j < kGJB; ++j)
      row[j] = (lane < b && j < b) ? X[(size_t)(p0 + lane) * n + p0 + j] : (lane == j ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < kGJB; ++k) {
      double pr[kGJB];
#pragma unroll
      for (int j = 0; j < kGJB; ++j) pr[j] = readlane_d(row[j], k);
      const double inv = 1.0 / pr[k];
      // row k: divided by the pivot; other rows: minus (their column-k entry / pivot) row k; the
      // new column k: 1 / pivot in row k, -(entry / pivot) elsewhere
      const double mult = lane == k ? 1.0 - inv : row[k] * inv;
#pragma unroll
      for (int j = 0; j < kGJB; ++j)
        if (j != k) row[j] = fma(-mult, pr[j], row[j]);
      row[k] = lane == k ? inv : -mult;
    }
    if (lane < kGJB) {
#pragma unroll
      for (int j = 0; j < kGJB; ++j) Pi[lane][j] = row[j];
    }
  } else {
    for (int e = tid - 64; e < kGJB * 64; e += 192) {
      const int k = e / 64, j = e % 64;
      Rr[k][j] = (k < b && c0 + j < n) ? X[(size_t)(p0 + k) * n + c0 + j] : 0.0;
    }
    for (int e = tid - 64; e < 64 * kGJB; e += 192) {
      const int i = e / kGJB, k = e % kGJB;
      Cs[i][k] = (k < b && r0 + i < n) ? X[(size_t)(r0 + i) * n + p0 + k] : 0.0;
    }
  }
  __syncthreads();
  // T = P^{-1} X[R, tile columns] on MFMA: wave w forms the 16 x 16 tiles (w >> 1, 2 (w & 1) + u);
  // rows of T past b are zero (P^{-1} is padded with identity rows, the staged rows are zero)
  {
    const int a0 = 16 * (w >> 1);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q0 = 16 * (2 * (w & 1) + u);
      v4d t = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < kGJB / 4; ++st)
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(Pi[a0 + lm][4 * st + lk], Rr[4 * st + lk][q0 + lm],
                                                 t, 0, 0, 0);
      const int col = c0 + q0 + lm;
      const bool pcol = col >= p0 && col < p0 + b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = a0 + lk + 4 * i;
        // the pivot columns of Y[R, :] are P^{-1} itself
        Ts[k][q0 + lm] = pcol ? (k < b ? Pi[k][col - p0] : 0.0) : t[i];
      }
    }
  }
  __syncthreads();
  v4d acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < kGJB / 4; ++st) {
    const double a = Cs[16 * w + lm][4 * st + lk];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ts[4 * st + lk][16 * q + lm], acc[q], 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = c0 + 16 * q + lm;
    if (col >= n) continue;
    const bool pcol = col >= p0 && col < p0 + b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = r0 + 16 * w + lk + 4 * i;
      if (row >= n) continue;
      const size_t at = (size_t)row * n + col;
      if (row >= p0 && row < p0 + b) Y[at] = Ts[row - p0][col - c0];
      else Y[at] = (pcol ? 0.0 : xt[q][i]) - acc[q][i];
    }
  }
}

__global__ void k_f32_to_f64(const float *__restrict__ x, double *__restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

// ---- vector kernels for GMRES ----
constexpr int kDotChunk = 4096;

// partial[v * nchunk + c] = sum over chunk c of Q[v][i] * w[i]
__global__ __launch_bounds__(256) void k_multi_dot(const double *__restrict__ Q, size_t ldq,
                                                   const double *__restrict__ w, size_t n,
                                                   double *__restrict__ partial, int nchunk) {
  const int c = blockIdx.x, v = blockIdx.y;
  const double *q = Q + (size_t)v * ldq;
  const size_t i0 = (size_t)c * kDotChunk, i1 = min(n, i0 + kDotChunk);
  double s = 0.0;
  for (size_t i = i0 + threadIdx.x; i < i1; i += 256) s = fma(q[i], w[i], s);
  __shared__ double red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)v * nchunk + c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_partials(const double *__restrict__ partial, int nvec, int nchunk,
                               double *__restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(size_t)v * nchunk + c];
  out[v] = s;
}

// w[i] -= sum_v coef[v] Q[v][i]
// y[i] = sum_v coef[v] Q[v][i]
__global__ void k_combine(const double *__restrict__ Q, size_t ldq, const double *__restrict__ coef,
                          int nvec, double *__restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int v = 0; v < nvec; ++v) s = fma(coef[v], Q[(size_t)v * ldq + i], s);
    y[i] = s;
  }
}

__global__ void k_scale_copy(const double *__restrict__ x, double a, double *__restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// Classical Gram-Schmidt update w -= sum_v c_v Q[v] with c_v the sum of the partial dot products
// partial[v][0..nchunk) of Q[v] and w (each block sums them into LDS first).  With norm_partial,
// each block also writes the sum of its updated w_i^2.
__global__ __launch_bounds__(256) void k_cgs_sub(const double *__restrict__ Q, size_t ldq,
                                                 const double *__restrict__ partial, int nchunk,
                                                 int nvec, double *__restrict__ w, size_t n,
                                                 double *__restrict__ norm_partial) {
  extern __shared__ double coef[];
  for (int v = threadIdx.x; v < nvec; v += blockDim.x) {
    double c = 0.0;
    for (int k = 0; k < nchunk; ++k) c += partial[(size_t)v * nchunk + k];
    coef[v] = c;
  }
  __syncthreads();
  double sq = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int v = 0; v < nvec; ++v) acc = fma(coef[v], Q[(size_t)v * ldq + i], acc);
    const double wi = w[i] - acc;
    w[i] = wi;
    sq = fma(wi, wi, sq);
  }
  if (norm_partial) {
    __shared__ double red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) norm_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

// Arnoldi step j on the device: column j of the Hessenberg matrix H (row-major, m columns) from
// the two Gram-Schmidt passes (partial sums p1, p2) and the norm (partials pn), the earlier Givens
// rotations applied to it, the new rotation, the rotated right-hand side g, 1 / ||w|| for the
// normalisation and the residual estimate |g_{j+1}| / beta in res[j], written straight into
// host memory (coherent pinned memory mapped into the device's address space).
__global__ __launch_bounds__(256) void k_arnoldi(double *__restrict__ H, int m, int j,
                                                 const double *__restrict__ p1,
                                                 const double *__restrict__ p2, int nchunk,
                                                 const double *__restrict__ pn, int npn,
                                                 double *__restrict__ cs, double *__restrict__ sn,
                                                 double *__restrict__ g, double beta,
                                                 double *__restrict__ inv_nn,
                                                 double *__restrict__ res) {
  // the column and the earlier rotations are staged in LDS (dynamic: 3 (j+1) doubles), so the
  // sequential rotation sweep of thread 0 runs at LDS latency
  extern __shared__ double sh[];
  double *hc = sh, *sc = sh + (j + 1), *ss = sc + (j + 1);
  __shared__ double red[4];
  for (int v = threadIdx.x; v <= j; v += blockDim.x) {
    double c = 0.0;
    for (int k = 0; k < nchunk; ++k) c += p1[(size_t)v * nchunk + k] + p2[(size_t)v * nchunk + k];
    hc[v] = c;
    if (v < j) {
      sc[v] = cs[v];
      ss[v] = sn[v];
    }
  }
  double sq = 0.0;
  for (int b = threadIdx.x; b < npn; b += blockDim.x) sq += pn[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double nn = sqrt(fmax(red[0] + red[1] + red[2] + red[3], 0.0));
    *inv_nn = nn > 0.0 ? 1.0 / nn : 0.0;
    double a = hc[0];
    for (int i = 0; i < j; ++i) {
      const double b = hc[i + 1];
      hc[i] = sc[i] * a + ss[i] * b;
      a = -ss[i] * a + sc[i] * b;
    }
    const double rr = hypot(a, nn);
    const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? nn / rr : 0.0;
    cs[j] = cj;
    sn[j] = sj;
    hc[j] = rr;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = cj * gj;
    res[j] = nn > 0.0 ? fabs(g[j + 1]) / beta : 0.0;
  }
  __syncthreads();
  for (int v = threadIdx.x; v <= j; v += blockDim.x) H[(size_t)v * m + j] = hc[v];
  if (threadIdx.x == 0) H[(size_t)(j + 1) * m + j] = 0.0;
}

// y = R^{-1} g for the first it columns of the rotated Hessenberg matrix (row-major, leading
// dimension m): the upper triangle and g staged in LDS (it <= kBacksubMax), then column by column,
// the updates of one column spread over the workgroup.
constexpr int kBacksubMax = 88;  // (it^2 + 2 it) doubles stay within 64 KiB of LDS
__global__ __launch_bounds__(256) void k_backsub(const double *__restrict__ R, int m,
                                                 const double *__restrict__ g, int it,
                                                 double *__restrict__ y) {
  extern __shared__ double sh[];
  double *Rs = sh, *gs = sh + (size_t)it * it, *ys = gs + it;
  for (int idx = threadIdx.x; idx < it * it; idx += blockDim.x) {
    const int i = idx / it, k = idx % it;
    Rs[idx] = k >= i ? R[(size_t)i * m + k] : 0.0;
  }
  for (int i = threadIdx.x; i < it; i += blockDim.x) gs[i] = g[i];
  __syncthreads();
  for (int i = it - 1; i >= 0; --i) {
    if (threadIdx.x == 0) ys[i] = gs[i] / Rs[(size_t)i * it + i];
    __syncthreads();
    const double yi = ys[i];
    for (int r = threadIdx.x; r < i; r += blockDim.x) gs[r] -= Rs[(size_t)r * it + i] * yi;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < it; i += blockDim.x) y[i] = ys[i];
}

__global__ void k_scale_dev(double *__restrict__ y, const double *__restrict__ a, size_t n) {
  const double f = *a;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] *= f;
}

__global__ void k_axpby(double a, const double *__restrict__ x, double b, double *__restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

inline int grid1d(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 8192); }

// ---- representation formula ----
// One workgroup per point (x, t), lanes over panels j.  With k = floor(t / h) and eps = t - k h,
// interval i = k - m (m >= 1) is seen at the time distances delta in [s_m - h/2, s_m + h/2],
// s_m = (m - 1/2) h + eps, and the current interval k at delta in [0, eps].  The time integrals
// of the heat kernel G and of the double-layer kernel (r . n_y) / (2 delta) G over an interval:
//   closed form (the current interval and m = 1, 2): differences of erfc(z) and of
//     D(z) = erfc(z) + 2 z e^{-z^2} / sqrt(pi),  z = rho / (2 sqrt(alpha delta));
//   Taylor form (m >= 3): the even series of the interval average around s_m,
//     int G = h (4 pi alpha s)^{-3/2} e^{-w} S_{3/2}(w),
//     int (r . n)/(2 delta) G = (r . n)/2 (4 pi alpha)^{-3/2} h s^{-5/2} e^{-w} S_{5/2}(w),
//     S_p(w) = sum_k eps_m^{2k} / (2k+1)! Q^p_{2k}(w),  w = rho^2 / (4 alpha s),  eps_m = h / (2 s),
//   truncated so that the dropped terms stay below ~6e-16 of the interval's scale (eps_m <=
//   1 / (2m - 1)).  Since (r . n)/(2 delta) G carries one more power 1/delta than G, termwise
//   Q^{5/2}_n = Q^{3/2}_n - (Q^{3/2}_n)' (the prime is d/dw), so S_{5/2} = S_{3/2} - S_{3/2}' and one
//   Horner sweep with the derivative gives both.  The workgroup tabulates the coefficients of
//   S_{3/2} in w for every m in LDS; each lane then walks (panel, m, node), reusing the interval's
//   data and coefficients for the 7 nodes of its panel.
constexpr int kReprClosed = 2;  // intervals m = 1, 2 behind the current one in closed form

__device__ __forceinline__ int repr_deg(int m) {
  return m < 4 ? 20 : m < 6 ? 16 : m < 8 ? 14 : m < 16 ? 12 : m < 32 ? 10 : 8;
}

// LDS offset of the table of interval m (m >= 3): [c_m, prefV_m, prefK_m, S_3/2 coefficients],
// deg(m) + 1 coefficients.
__device__ __forceinline__ int repr_off(int m) {
  int off = 0;
  const int lo[6] = {3, 4, 6, 8, 16, 32}, hi[6] = {4, 6, 8, 16, 32, 1 << 30};
  const int deg[6] = {20, 16, 14, 12, 10, 8};
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int n = max(0, min(m, hi[c]) - lo[c]);
    off += n * (3 + deg[c] + 1);
  }
  return off;
}

// Intervals m = mlo .. mhi-1 of one degree class (polynomial length N) for panel j: adds the
// panel's single-layer sum (weights w, before the panel's area) to ps and its double-layer sum
// (data g at the panel's vertices) to pd.
template <int N>
__device__ __forceinline__ void repr_taylor(const AsmParams &p, const double *__restrict__ tab,
                                            const double *__restrict__ w,
                                            const double *__restrict__ g, int k, int mlo, int mhi,
                                            int j, int v0, int v1, int v2,
                                            const double (&r2)[kFarN], const double (&rn)[kFarN],
                                            const double *etab, double &ps, double &pd) {
  const int ne = p.ne, nv = p.nv;
  const double *T = tab + repr_off(mlo);
#pragma unroll 1
  for (int m = mlo; m < mhi; ++m, T += 3 + N) {
    const double cm = T[0];
    const int i = k - m;
    const double wi = w[(size_t)i * ne + j] * T[1];
    const double *gi = g + (size_t)i * nv;
    const double pk = T[2];
    const double g0 = gi[v0], g1 = gi[v1], g2 = gi[v2];
    double c[N];
#pragma unroll
    for (int n = 0; n < N; ++n) c[n] = T[3 + n];
    double sV = 0.0, sK0 = 0.0, sK1 = 0.0, sK2 = 0.0;
#pragma unroll
    for (int q = 0; q < kFarN; ++q) {
      const double x = r2[q] * cm;
      const double ew = exp_neg_m(x, etab) * p.w7[q];
      double P, dP;
      horner_d<N>(c, x, P, dP);
      sV = fma(ew, P, sV);
      const double u = ew * rn[q] * (P - dP);
      sK0 = fma(p.lam7[q][0], u, sK0);
      sK1 = fma(p.lam7[q][1], u, sK1);
      sK2 = fma(p.lam7[q][2], u, sK2);
    }
    ps = fma(wi, sV, ps);
    pd = fma(pk, fma(g0, sK0, fma(g1, sK1, g2 * sK2)), pd);
  }
}

__global__ __launch_bounds__(256, 2) void k_repr(const AsmParams *__restrict__ pp,
                                              const double *__restrict__ qtab,
                                              const double *__restrict__ pts,
                                              const double *__restrict__ w,
                                              const double *__restrict__ g,
                                              double *__restrict__ u, double *__restrict__ sl,
                                              double *__restrict__ dl) {
  extern __shared__ double tab[];
  const AsmParams &p = *pp;
  const int pid = blockIdx.x;
  const double px = pts[4 * pid], py = pts[4 * pid + 1], pz = pts[4 * pid + 2], t = pts[4 * pid + 3];
  const int ne = p.ne, nv = p.nv, nt = p.nt;
  const double h = p.h, al = p.alpha;
  int k = (int)floor(t / h);
  k = max(0, min(k, nt));
  double eps = t - k * h;
  if (eps < 0.0) eps = 0.0;
  constexpr double kPi = 3.14159265358979323846;
  __shared__ double etab[kExpTabN];
  stage_exp_tab_pos(etab);
  // the series' coefficient table Q, staged once per workgroup
  constexpr int kQn = kReprQ * (kReprDeg + 1);
  __shared__ double qs[kQn];
  for (int i = threadIdx.x; i < kQn; i += blockDim.x) qs[i] = qtab[i];
  __syncthreads();
  // per-interval tables: one thread per (interval m, coefficient), so that the long tables of
  // the near intervals are spread over the workgroup
  constexpr int kItems = kReprDeg + 1;
  const int nitems = max(0, k - kReprClosed) * kItems;
  for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
    const int m = kReprClosed + 1 + it / kItems;
    const int jj = it % kItems;
    const int D = repr_deg(m);
    if (jj > D) continue;
    double *T = tab + repr_off(m);
    const double sm = (m - 0.5) * h + eps;
    const double em = h / (2.0 * sm), e2 = em * em;
    if (jj == 0) {
      T[0] = 1.0 / (4.0 * al * sm);
      T[1] = 4.0 * kPi * al * h * pow(4.0 * kPi * al * sm, -1.5);
      T[2] = 2.0 * kPi * pow(4.0 * kPi * al, -1.5) * h * pow(sm, -2.5);
    }
    double c = 0.0;
    for (int kk = D / 2; kk >= 0; --kk) c = fma(c, e2, 2 * kk >= jj ? qs[kk * (kReprDeg + 1) + jj] : 0.0);
    T[3 + jj] = c;
  }
  __syncthreads();

  const double c_al = 1.0 / (2.0 * sqrt(al));
  constexpr double kTwoInvSqrtPi = 1.1283791670955125739;
  // z = rho cz[m] at the closed-form levels: the current interval (time distance eps) and the
  // intervals m = 1 .. kReprClosed behind it (m h + eps); the same for every panel of the point
  double cz[kReprClosed + 1];
  cz[0] = eps > 0.0 ? c_al / sqrt(eps) : 0.0;
#pragma unroll
  for (int m = 1; m <= kReprClosed; ++m) cz[m] = c_al / sqrt(m * h + eps);
  double accs = 0.0, accd = 0.0;
  for (int j = threadIdx.x; j < ne; j += blockDim.x) {
    const double area = p.geom[24 * ne + j];
    const double n0 = p.geom[21 * ne + j], n1 = p.geom[22 * ne + j], n2 = p.geom[23 * ne + j];
    const int v0 = p.tris[3 * j], v1 = p.tris[3 * j + 1], v2 = p.tris[3 * j + 2];
    double r2[kFarN], rn[kFarN];
#pragma unroll
    for (int q = 0; q < kFarN; ++q) {
      const double rx = px - p.geom[(q * 3 + 0) * ne + j];
      const double ry = py - p.geom[(q * 3 + 1) * ne + j];
      const double rz = pz - p.geom[(q * 3 + 2) * ne + j];
      r2[q] = fma(rx, rx, fma(ry, ry, rz * rz));
      const double rho = sqrt(r2[q]);
      rn[q] = fma(rx, n0, fma(ry, n1, rz * n2));
      const double Wq = p.w7[q] * area;
      // closed form: current interval and m = 1 .. min(k, kReprClosed)
      const double l0 = p.lam7[q][0], l1 = p.lam7[q][1], l2 = p.lam7[q][2];
      double sv = 0.0, sd = 0.0, ec_prev = 0.0, D_prev = 0.0;
      if (eps > 0.0) {
        const double z = rho * cz[0];
        ec_prev = erfc(z);
        D_prev = ec_prev + kTwoInvSqrtPi * z * exp_neg(z * z);
        if (k < nt) {
          sv += w[(size_t)k * ne + j] * ec_prev;
          const double *gk = g + (size_t)k * nv;
          sd += (l0 * gk[v0] + l1 * gk[v1] + l2 * gk[v2]) * D_prev;
        }
      }
      const int mc = min(k, kReprClosed);
#pragma unroll
      for (int m = 1; m <= kReprClosed; ++m) {
        if (m > mc) break;
        const double z = rho * cz[m];
        const double ec = erfc(z);
        const double D = ec + kTwoInvSqrtPi * z * exp_neg(z * z);
        const int i = k - m;
        sv += w[(size_t)i * ne + j] * (ec - ec_prev);
        const double *gi = g + (size_t)i * nv;
        sd += (l0 * gi[v0] + l1 * gi[v1] + l2 * gi[v2]) * (D - D_prev);
        ec_prev = ec;
        D_prev = D;
      }
      const double ir = 1.0 / rho;
      accs = fma(Wq * ir, sv, accs);
      accd = fma(Wq * rn[q] * (ir * ir * ir), sd, accd);
    }
    // Taylor form for m = 3 .. k, by degree class
    const int m0 = kReprClosed + 1;
    double ps = 0.0, pd = 0.0;
    repr_taylor<21>(p, tab, w, g, k, m0, min(k + 1, 4), j, v0, v1, v2, r2, rn, etab, ps, pd);
    repr_taylor<17>(p, tab, w, g, k, 4, min(k + 1, 6), j, v0, v1, v2, r2, rn, etab, ps, pd);
    repr_taylor<15>(p, tab, w, g, k, 6, min(k + 1, 8), j, v0, v1, v2, r2, rn, etab, ps, pd);
    repr_taylor<13>(p, tab, w, g, k, 8, min(k + 1, 16), j, v0, v1, v2, r2, rn, etab, ps, pd);
    repr_taylor<11>(p, tab, w, g, k, 16, min(k + 1, 32), j, v0, v1, v2, r2, rn, etab, ps, pd);
    repr_taylor<9>(p, tab, w, g, k, 32, k + 1, j, v0, v1, v2, r2, rn, etab, ps, pd);
    accs = fma(area, ps, accs);
    accd = fma(area, pd, accd);
  }
  __shared__ double red[2][4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    accs += __shfl_xor(accs, o, 64);
    accd += __shfl_xor(accd, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = accs;
    red[1][threadIdx.x >> 6] = accd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr double kInv4Pi = 0.079577471545947667884;
    const double s = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) * kInv4Pi / p.alpha;
    const double d = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) * kInv4Pi;
    u[pid] = s - d;
    if (sl) sl[pid] = s;
    if (dl) dl[pid] = d;
  }
}

// Potentials on a non-uniform time grid t_0 = 0 < ... < t_{E_t} (the paper's outlook, Sec. 7, with
// the time integrals of Sec. 3.5 over general intervals): one workgroup per point (x, t), lanes
// over panels.  With t_k <= t < t_{k+1}, interval i < k is seen at s = t - tau in
// [t - t_{i+1}, t - t_i] and the current interval k at [0, t - t_k]; every interval in closed form
// (differences of erfc and of D(z) = erfc(z) + 2 z e^{-z^2} / sqrt(pi) at its two ends, each end's
// values shared by the two intervals that meet there).  The breakpoint factors
// 1 / (2 sqrt(alpha (t - t_b))) sit in LDS; a lane walks its panel's breakpoints from t back to 0
// and carries the previous end's values per rule node.
__global__ __launch_bounds__(256) void k_nu_repr(const AsmParams *__restrict__ pp,
                                                 const double *__restrict__ tn,
                                                 const double *__restrict__ pts,
                                                 const double *__restrict__ w,
                                                 const double *__restrict__ g,
                                                 double *__restrict__ u, double *__restrict__ sl,
                                                 double *__restrict__ dl) {
  extern __shared__ double czs[];  // [E_t + 1]: 1 / (2 sqrt(alpha (t - t_b))), 0 where t = t_b
  const AsmParams &p = *pp;
  const int pid = blockIdx.x;
  const double px = pts[4 * pid], py = pts[4 * pid + 1], pz = pts[4 * pid + 2], t = pts[4 * pid + 3];
  const int ne = p.ne, nv = p.nv, nt = p.nt;
  // k: the largest index <= E_t with t_k <= t (t_0 = 0 <= t)
  int lo = 0, hi = nt;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tn[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const int k = lo;
  const double c_al = 1.0 / (2.0 * sqrt(p.alpha));
  for (int b = threadIdx.x; b <= k; b += blockDim.x) {
    const double s = t - tn[b];
    czs[b] = s > 0.0 ? c_al / sqrt(s) : 0.0;
  }
  __syncthreads();
  constexpr double kTwoInvSqrtPi = 1.1283791670955125739;
  double accs = 0.0, accd = 0.0;
  for (int j = threadIdx.x; j < ne; j += blockDim.x) {
    const double area = p.geom[24 * ne + j];
    const double n0 = p.geom[21 * ne + j], n1 = p.geom[22 * ne + j], n2 = p.geom[23 * ne + j];
    const int v0 = p.tris[3 * j], v1 = p.tris[3 * j + 1], v2 = p.tris[3 * j + 2];
    double rho[kFarN], rn[kFarN], ecp[kFarN], Dp[kFarN], sv[kFarN], sd[kFarN];
#pragma unroll
    for (int q = 0; q < kFarN; ++q) {
      const double rx = px - p.geom[(q * 3 + 0) * ne + j];
      const double ry = py - p.geom[(q * 3 + 1) * ne + j];
      const double rz = pz - p.geom[(q * 3 + 2) * ne + j];
      rho[q] = sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
      rn[q] = fma(rx, n0, fma(ry, n1, rz * n2));
      ecp[q] = Dp[q] = sv[q] = sd[q] = 0.0;  // the values at s = 0
    }
#pragma unroll 1
    for (int b = k; b >= 0; --b) {
      const double cz = czs[b];
      // interval b ends at this breakpoint (none for b = E_t)
      const bool has = b < nt;
      const double wb = has ? w[(size_t)b * ne + j] : 0.0;
      const double *gb = g + (size_t)(has ? b : 0) * nv;
      const double g0 = has ? gb[v0] : 0.0, g1 = has ? gb[v1] : 0.0, g2 = has ? gb[v2] : 0.0;
#pragma unroll
      for (int q = 0; q < kFarN; ++q) {
        double ec = 0.0, D = 0.0;
        if (cz > 0.0) {
          const double z = rho[q] * cz;
          ec = erfc(z);
          D = ec + kTwoInvSqrtPi * z * exp_neg(z * z);
        }
        sv[q] = fma(wb, ec - ecp[q], sv[q]);
        const double gq = fma(p.lam7[q][0], g0, fma(p.lam7[q][1], g1, p.lam7[q][2] * g2));
        sd[q] = fma(gq, D - Dp[q], sd[q]);
        ecp[q] = ec;
        Dp[q] = D;
      }
    }
#pragma unroll
    for (int q = 0; q < kFarN; ++q) {
      const double Wq = p.w7[q] * area, ir = 1.0 / rho[q];
      accs = fma(Wq * ir, sv[q], accs);
      accd = fma(Wq * rn[q] * (ir * ir * ir), sd[q], accd);
    }
  }
  __shared__ double red[2][4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    accs += __shfl_xor(accs, o, 64);
    accd += __shfl_xor(accd, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = accs;
    red[1][threadIdx.x >> 6] = accd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr double kInv4Pi = 0.079577471545947667884;
    const double s = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) * kInv4Pi / p.alpha;
    const double d = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) * kInv4Pi;
    u[pid] = s - d;
    if (sl) sl[pid] = s;
    if (dl) dl[pid] = d;
  }
}

// ------------------------------------------------------------------------------------------
// host helpers
// ------------------------------------------------------------------------------------------
int ensure_work(hb_ctx *c, size_t bytes) {
  if (c->work_bytes >= bytes) return HB_OK;
  if (c->d_work) (void)hipFree(c->d_work);
  c->d_work = nullptr;
  c->work_bytes = 0;
  HB_CHECK(c, hipMalloc(&c->d_work, bytes));
  c->work_bytes = bytes;
  return HB_OK;
}

}  // namespace

// y = A x (Toeplitz), y overwritten
// Split of the product over workgroups: 64-row tiles x column groups (cpg chunks each) x d
// slices (slice z takes every slices-th block from dlo + z, so all slices carry the same work),
// aiming at >= kApplyWant workgroups with as few partial results as possible.
constexpr int kApplyWant = 768;
struct ApplySplit {
  int rt, nchunk, cpg, groups, slices;
};

// max_parts > 0 caps groups x slices (the partial results held at once); slices go first.
static ApplySplit apply_split(int R, int C, int nd, int max_parts = 0) {
  ApplySplit a;
  a.rt = (R + TR - 1) / TR;
  a.nchunk = (C + kTC - 1) / kTC;
  const int want = kApplyWant;
  int groups = std::max(1, std::min(a.nchunk, (want + a.rt - 1) / a.rt));
  if (max_parts > 0) groups = std::min(groups, max_parts);
  a.cpg = (a.nchunk + groups - 1) / groups;
  a.groups = (a.nchunk + a.cpg - 1) / a.cpg;
  a.slices = std::max(1, std::min(std::max(1, nd / 8), (want + a.rt * a.groups - 1) / (a.rt * a.groups)));
  if (max_parts > 0) a.slices = std::max(1, std::min(a.slices, max_parts / a.groups));
  return a;
}

// ------------------------------------------------------------------------------------------
// Fixed scratch of hb_apply_noalloc: the partial results of the product live in this array
// instead of a buffer the context allocates.  Each device holds its own copy at its own address,
// looked up once per device (hipGetSymbolAddress, at context creation) and used through that
// address only; the array's name is not a device address in host code.
// ------------------------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// Y[k] = sum_{d in [dlo, dhi)} A^d X[k - d] with X restricted to the times [jlo, jhi); with sub,
// y[k] -= Y[k] for ksub <= k < khi (khi < 0: E_t) instead of y = Y.  ntw > 0: x and y hold a
// window of ntw time steps (the product sees no earlier times).
// scratch / scratch_bytes: caller-provided room for the partial results (no allocation; the split
// is narrowed to fit, HB_EINVAL if one part does not fit); NULL: the context's own buffer.
template <typename TA>
static int launch_toeplitz(hb_ctx *c, const TA *A, int R, int C, const double *x, double *y,
                           hipStream_t s, int dlo, int dhi, int jlo, int jhi, bool sub, int ksub,
                           void *scratch_buf = nullptr, size_t scratch_bytes = 0, int khi = -1,
                           int ntw = -1) {
  const int nt = ntw > 0 ? ntw : c->nt;
  const int klo = sub ? ksub : 0;
  if (khi < 0 || !sub) khi = nt;
  if (nt > 256) {
    c->err = "toeplitz apply supports E_t <= 256";
    return HB_EINVAL;
  }
  const int nd = std::max(0, dhi - dlo);
  const size_t ny = (size_t)nt * R;
  int max_parts = 0;
  if (scratch_buf) {
    const size_t fit = scratch_bytes / (sizeof(TA) * ny);
    if (fit < 1) {
      c->err = "block-Toeplitz partial results (E_t x rows x element size) exceed the fixed scratch";
      return HB_EINVAL;
    }
    max_parts = (int)std::min<size_t>(fit, 1 << 20);
  }
  if (nd == 0) {
    if (!sub) hipLaunchKernelGGL(k_fill, dim3(grid1d((size_t)nt * R)), dim3(256), 0, s, y, (size_t)nt * R, 0.0);
    return HB_OK;
  }
  const ApplySplit sp = apply_split(R, C, nd, max_parts);
  const int parts = sp.groups * sp.slices;
  const size_t need = sizeof(TA) * ny * parts;
  TA *P;
  if (scratch_buf) {
    P = (TA *)scratch_buf;
  } else {
    if (c->apply_bytes < need) {
      if (c->d_apply) (void)hipFree(c->d_apply);
      c->d_apply = nullptr;
      c->apply_bytes = 0;
      HB_CHECK(c, hipMalloc(&c->d_apply, need));
      c->apply_bytes = need;
    }
    P = (TA *)c->d_apply;
  }
  int ntc = 1;
  while (ntc * 16 < nt) ntc *= 2;
  dim3 grid(sp.rt, sp.groups, sp.slices);
#define HB_TOEP(NTC_)                                                                          \
  hipLaunchKernelGGL((k_toeplitz<TA, NTC_>), grid, dim3(256), 0, s, A, x, P, nt, R, C, sp.cpg, \
                     dlo, dhi, jlo, jhi, klo, khi)
  switch (ntc) {
    case 1: HB_TOEP(1); break;
    case 2: HB_TOEP(2); break;
    case 4: HB_TOEP(4); break;
    case 8: HB_TOEP(8); break;
    default: HB_TOEP(16); break;
  }
#undef HB_TOEP
  if (khi > klo)
    hipLaunchKernelGGL(k_sum_groups<TA>, dim3(grid1d((size_t)(khi - klo) * R)), dim3(256), 0, s, P,
                       parts, ny, y, sub ? 1 : 0, (size_t)klo * R, (size_t)khi * R);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

int toeplitz_apply(hb_ctx *c, const void *blocks, int R, int C, const double *x, double *y,
                   hipStream_t s) {
  const int nt = c->nt;
  if (c->storage_f32)
    return launch_toeplitz<float>(c, (const float *)blocks, R, C, x, y, s, 0, nt, 0, nt, false, 0);
  return launch_toeplitz<double>(c, (const double *)blocks, R, C, x, y, s, 0, nt, 0, nt, false, 0);
}

int toeplitz_apply32(hb_ctx *c, const float *blocks, int R, int C, const double *x, double *y,
                     hipStream_t s) {
  return launch_toeplitz<float>(c, blocks, R, C, x, y, s, 0, c->nt, 0, c->nt, false, 0);
}

// Block lower-triangular product on a non-uniform grid: y^k[r] = sum_{i <= k} sum_c A^{k,i}[r][c]
// x^i[c], blocks packed [k (k + 1) / 2 + i][R][C].  Every block is read once (no Toeplitz reuse),
// so the product streams the blocks from HBM: one wave per row r of block row k, the lanes over
// the columns of each block of the row (coalesced), four independent partial sums per lane, then
// a wave reduction.  Long block rows are launched first.
__global__ __launch_bounds__(256) void k_nu_apply(const double *__restrict__ A,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ y, int nt, int R, int C) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + w;
  const int k = nt - 1 - (int)blockIdx.y;
  if (r >= R) return;
  const size_t blk = (size_t)R * C;
  const double *a = A + ((size_t)k * (k + 1) / 2) * blk + (size_t)r * C;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int i = 0; i <= k; ++i, a += blk) {
    const double *xi = x + (size_t)i * C;
    int c = lane;
    for (; c + 192 < C; c += 256) {
      s0 = fma(a[c], xi[c], s0);
      s1 = fma(a[c + 64], xi[c + 64], s1);
      s2 = fma(a[c + 128], xi[c + 128], s2);
      s3 = fma(a[c + 192], xi[c + 192], s3);
    }
    for (; c < C; c += 64) s0 = fma(a[c], xi[c], s0);
  }
  double sum = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) y[(size_t)k * R + r] = sum;
}

// Time marching on a non-uniform grid, the history of step k: r^k -= sum_{i<k} V^{k,i} w^i over
// the block row k (packed blocks k (k + 1) / 2 .. k (k + 1) / 2 + k - 1, consecutive), one wave
// per row, kGemvBatch column loads of a round in flight per lane.
__global__ __launch_bounds__(256) void k_nu_hist(const double *__restrict__ A,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ r, int k, int R, int C) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= R) return;
  const size_t blk = (size_t)R * C;
  const double *a = A + ((size_t)k * (k + 1) / 2) * blk + (size_t)row * C;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < k; ++i, a += blk) {
    const double *xi = x + (size_t)i * C;
    for (int c0 = 0; c0 < C; c0 += 64 * kGemvBatch) {
      double av[kGemvBatch], xv[kGemvBatch];
#pragma unroll
      for (int u = 0; u < kGemvBatch; ++u) {
        const int c = c0 + lane + 64 * u;
        av[u] = c < C ? a[c] : 0.0;
        xv[u] = c < C ? xi[c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGemvBatch; ++u) s[u & 3] = fma(av[u], xv[u], s[u & 3]);
    }
  }
  double t = (s[0] + s[1]) + (s[2] + s[3]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (lane == 0) r[(size_t)k * R + row] -= t;
}

int nu_apply(hb_ctx *c, const double *A, int R, int C, const double *x, double *y, hipStream_t s) {
  dim3 grid((unsigned)((R + 3) / 4), (unsigned)c->nt);
  hipLaunchKernelGGL(k_nu_apply, grid, dim3(256), 0, s, A, x, y, c->nt, R, C);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

// Address of this device's copy of `scratch`, looked up once per device with that device current.
int static_scratch_init(hb_ctx *c) {
  if (c->device < 0 || c->device >= kMaxDevices) {
    c->err = "device index beyond the fixed-scratch table";
    return HB_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[c->device]) return HB_OK;
  void *ptr = nullptr;
  HB_CHECK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) {
    c->err = "hipGetSymbolAddress returned no address for the fixed scratch";
    return HB_EHIP;
  }
  g_scratch_ptr[c->device] = ptr;
  return HB_OK;
}

static void *static_scratch(const hb_ctx *c) {
  if (c->device < 0 || c->device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[c->device];
}

namespace {

// out[(k0 + d) * R + row] = beta * out + alpha * (A^{d_first + d} x), d = 0 .. nd-1
int gemv_batch(hb_ctx *c, const void *A, size_t stride, int R, int C, int nd, const double *x,
               double *out, double alpha, double beta, size_t out_stride, hipStream_t s) {
  if (nd <= 0) return HB_OK;
  dim3 grid((R + 3) / 4, nd);
  if (c->storage_f32 && A != (const void *)c->d_v0inv)
    hipLaunchKernelGGL(k_gemv_rows<float>, grid, dim3(256), 0, s, (const float *)A, stride, x, out,
                       R, C, alpha, beta, out_stride);
  else
    hipLaunchKernelGGL(k_gemv_rows<double>, grid, dim3(256), 0, s, (const double *)A, stride, x,
                       out, R, C, alpha, beta, out_stride);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

// Inverse of the n x n double matrix held in A (overwritten by the inverse) by blocked
// Gauss-Jordan elimination without pivoting (A is V_h^0 or a mass matrix, both symmetric positive
// definite); B: an n x n workspace.  The panels alternate between A and B; with an odd panel count
// the matrix is first copied to B so that the last panel writes A.
int gj_invert(hb_ctx *c, double *A, double *B, int n, hipStream_t s, int nmat = 1) {
  // nmat > 1: a batch of nmat matrices n * n doubles apart in A (and in B), inverted together
  const dim3 tiles((n + 63) / 64, (n + 63) / 64, nmat);
  const size_t zs = (size_t)n * n;
  const int panels = (n + kGJB - 1) / kGJB;
  double *X = A, *Y = B;
  if (panels & 1) {
    HB_CHECK(c, hipMemcpyAsync(B, A, sizeof(double) * zs * nmat, hipMemcpyDeviceToDevice, s));
    std::swap(X, Y);
  }
  for (int p0 = 0; p0 < n; p0 += kGJB) {
    hipLaunchKernelGGL(k_gj_step, tiles, dim3(256), 0, s, X, Y, n, p0, std::min(kGJB, n - p0), zs);
    std::swap(X, Y);
  }
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

int invert_v0(hb_ctx *c, hipStream_t s) {
  if (c->v0inv_valid) return HB_OK;
  const int n = (int)c->ne;
  const size_t nn = (size_t)n * n;
  if (c->nu) {
    // every diagonal block V^{k,k} (packed index k (k + 1) / 2 + k), inverted as one batch
    const int nt = c->nt;
    if (!c->d_v0inv) HB_CHECK(c, hipMalloc(&c->d_v0inv, sizeof(double) * 2 * nn * nt));
    double *A = c->d_v0inv, *B = A + nn * nt;
    for (int k = 0; k < nt; ++k)
      HB_CHECK(c, hipMemcpyAsync(A + (size_t)k * nn, (const double *)c->d_V + ((size_t)k * (k + 1) / 2 + k) * nn,
                                 sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    int rc = gj_invert(c, A, B, n, s, nt);
    if (rc) return rc;
    c->v0inv_valid = true;
    return HB_OK;
  }
  if (!c->d_v0inv) HB_CHECK(c, hipMalloc(&c->d_v0inv, sizeof(double) * 2 * nn));
  double *A = c->d_v0inv, *B = A + nn;
  if (c->storage_f32)
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid1d(nn)), dim3(256), 0, s, (const float *)c->d_V, A, nn);
  else
    HB_CHECK(c, hipMemcpyAsync(A, c->d_V, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
  int rc = gj_invert(c, A, B, n, s);
  if (rc) return rc;
  c->v0inv_valid = true;
  return HB_OK;
}

// Inverse of the p1 mass matrix M[i][j] = int phi^1_i phi^1_j (sum over the panels at i and j of
// area (1 + [i == j]) / 12), formed once per context; the operator preconditioner of the
// Neumann system applies M_h^{-1} = (h M)^{-1} in every time step.
int ensure_minv(hb_ctx *c, hipStream_t s) {
  if (c->minv_valid) return HB_OK;
  const int n = (int)c->nv;
  const size_t nn = (size_t)n * n;
  // inverse, then kBlockPad zero bytes (read by the Toeplitz product's fragment loads), then the
  // elimination's second buffer
  const size_t padn = kBlockPad / sizeof(double);
  if (!c->d_minv) HB_CHECK(c, hipMalloc(&c->d_minv, sizeof(double) * (2 * nn + padn)));
  std::vector<double> M(nn, 0.0);
  for (int64_t t = 0; t < c->ne; ++t)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        M[(size_t)c->tris[3 * t + a] * n + c->tris[3 * t + b]] += c->area[t] * (a == b ? 2.0 : 1.0) / 12.0;
  double *A = c->d_minv, *B = A + nn + padn;
  HB_CHECK(c, hipMemcpyAsync(A, M.data(), sizeof(double) * nn, hipMemcpyHostToDevice, s));
  int rc = gj_invert(c, A, B, n, s);
  if (rc) return rc;
  HB_CHECK(c, hipMemsetAsync(A + nn, 0, kBlockPad, s));
  HB_CHECK(c, hipGetLastError());
  HB_CHECK(c, hipStreamSynchronize(s));  // M lives on the host stack
  c->minv_valid = true;
  return HB_OK;
}

// dots out[v] = Q_v . w for v < nvec (device), copied to host hv
int multi_dot(hb_ctx *c, const double *Q, size_t ldq, int nvec, const double *w, size_t n,
              double *partial, double *dres, double *hv, hipStream_t s) {
  const int nchunk = (int)((n + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(k_multi_dot, dim3(nchunk, nvec), dim3(256), 0, s, Q, ldq, w, n, partial, nchunk);
  hipLaunchKernelGGL(k_sum_partials, dim3((nvec + 255) / 256), dim3(256), 0, s, partial, nvec, nchunk, dres);
  HB_CHECK(c, hipMemcpyAsync(hv, dres, sizeof(double) * nvec, hipMemcpyDeviceToHost, s));
  HB_CHECK(c, hipStreamSynchronize(s));
  return HB_OK;
}

}  // namespace

}  // namespace hb

using namespace hb;

namespace {

int ctx_fail(hb_ctx *c, int code, const std::string &m) {
  if (c) c->err = m;
  return code;
}

// Workspace layout for the solvers (doubles):
//   GMRES: Q[(m+1) n] | r[n] | partial[(m+1) * nchunk] | dres[m+1] | coef[m+1]
// V_h x with the double blocks (op 0) or with the float copy on the float MFMA path (op 1);
// op 2: D_h x (the Neumann system)
int apply_V(hb_ctx *c, int op, const double *x, double *y, hipStream_t s) {
  if (op == 0 && c->nu) return nu_apply(c, (const double *)c->d_V, (int)c->ne, (int)c->ne, x, y, s);
  if (op == 0) return toeplitz_apply(c, c->d_V, (int)c->ne, (int)c->ne, x, y, s);
  if (op == 2) return toeplitz_apply(c, c->d_D, (int)c->nv, (int)c->nv, x, y, s);
  const float *V32 = c->storage_f32 ? (const float *)c->d_V : c->d_V32;
  return toeplitz_apply32(c, V32, (int)c->ne, (int)c->ne, x, y, s);
}

int ensure_V32(hb_ctx *c, hipStream_t s) {
  if (c->storage_f32 || c->V32_valid) return HB_OK;
  const size_t n = (size_t)c->nt * c->ne * c->ne;
  if (!c->d_V32) {
    HB_CHECK(c, hipMalloc(&c->d_V32, n * sizeof(float) + kBlockPad));
    HB_CHECK(c, hipMemsetAsync((char *)c->d_V32 + n * sizeof(float), 0, kBlockPad, s));
  }
  hipLaunchKernelGGL(k_to_float, dim3(grid1d(n)), dim3(256), 0, s, (const double *)c->d_V, c->d_V32, n);
  HB_CHECK(c, hipGetLastError());
  c->V32_valid = true;
  return HB_OK;
}

// Operator preconditioner of the Neumann system (the paper's use of V_h^{11}, Sec. 6.1):
// z = M_h^{-1} V_h^{11} M_h^{-1} q with M_h = h blockdiag(M), M the p1 mass matrix.
int op_precond_apply(hb_ctx *c, const double *q, double *z, hipStream_t s) {
  const size_t n = (size_t)c->nt * c->nv;
  if (!c->d_pcw || c->pcw_n < n) {
    if (c->d_pcw) (void)hipFree(c->d_pcw);
    c->d_pcw = nullptr;
    c->pcw_n = 0;
    HB_CHECK(c, hipMalloc(&c->d_pcw, sizeof(double) * 2 * n));
    c->pcw_n = n;
  }
  double *t1 = c->d_pcw, *t2 = t1 + n;
  const int nv = (int)c->nv, nt = c->nt;
  int rc = launch_toeplitz<double>(c, c->d_minv, nv, nv, q, t1, s, 0, 1, 0, nt, false, 0);
  if (rc) return rc;
  if ((rc = toeplitz_apply(c, c->d_V11, nv, nv, t1, t2, s))) return rc;
  if ((rc = launch_toeplitz<double>(c, c->d_minv, nv, nv, t2, z, s, 0, 1, 0, nt, false, 0))) return rc;
  hipLaunchKernelGGL(k_axpby, dim3(grid1d(n)), dim3(256), 0, s, 1.0 / (c->h * c->h), z, 0.0, z, n);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

// z = P q: 1 the learned block-diagonal map (V_h), 2 the operator preconditioner (D_h)
int pc_apply(hb_ctx *c, int kind, const double *q, double *z, hipStream_t s) {
  return kind == 2 ? op_precond_apply(c, q, z, s) : precond_apply(c, q, z, s);
}

// Unrestarted GMRES (right-preconditioned by the learned block-diagonal map when precond) with
// classical Gram-Schmidt applied twice.  The Arnoldi recurrence (Hessenberg column, Givens
// rotations, residual estimate) stays on the device; the host learns each step's residual
// estimate one step late through pinned memory while the next step is already queued, so the GPU
// never waits for the host; when the estimate extrapolated from the last two steps says that the
// step in flight may be the last, the host waits for it instead of queueing a surplus step.
// bnorm: ||b|| when the caller has it (computed as here: the dot kernels, then sqrt), else < 0
int gmres(hb_ctx *c, int op, const double *b, double *x, double tol, int maxit, hipStream_t s,
          hb_solve_info *info, int precond = 0, double bnorm = -1.0) {
  const size_t n = (size_t)c->nt * (op == 2 ? c->nv : c->ne);
  const int m = maxit;
  const int nchunk = (int)((n + kDotChunk - 1) / kDotChunk);
  const int nblk = grid1d(n);
  const size_t need = sizeof(double) * ((size_t)(m + 1) * n + n + 2 * (size_t)(m + 1) * nchunk +
                                        nblk + (size_t)(m + 1) * m + 4 * (size_t)(m + 1) + 4);
  int rc = ensure_work(c, need);
  if (rc) return rc;
  double *Q = c->d_work, *r = Q + (size_t)(m + 1) * n;  // r: P q_j
  double *p1 = r + n, *p2 = p1 + (size_t)(m + 1) * nchunk, *pn = p2 + (size_t)(m + 1) * nchunk;
  double *dH = pn + nblk, *dcs = dH + (size_t)(m + 1) * m, *dsn = dcs + (m + 1);
  double *dg = dsn + (m + 1), *dres = dg + (m + 1), *dinv = dres + (m + 1);
  if (!c->h_res || c->h_res_n < m + 1) {
    if (c->h_res) (void)hipHostFree(c->h_res);
    c->h_res = nullptr;
    c->h_res_n = 0;
    HB_CHECK(c, hipHostMalloc((void **)&c->h_res, sizeof(double) * (m + 1),
                              hipHostMallocMapped | hipHostMallocCoherent));
    c->h_res_n = m + 1;
  }
  double *res_dev = nullptr;  // the device's address of h_res
  HB_CHECK(c, hipHostGetDevicePointer((void **)&res_dev, c->h_res, 0));
  if (!c->ev_step) HB_CHECK(c, hipEventCreateWithFlags(&c->ev_step, hipEventDisableTiming));
  if (!c->ev_prev) HB_CHECK(c, hipEventCreateWithFlags(&c->ev_prev, hipEventDisableTiming));
  double beta = bnorm;
  if (beta < 0.0) {
    std::vector<double> tmp(1);
    if ((rc = multi_dot(c, b, 0, 1, b, n, p1, dres, tmp.data(), s))) return rc;
    beta = std::sqrt(tmp[0]);
  }
  if (beta == 0.0) {
    hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(256), 0, s, x, n, 0.0);
    if (info) { info->iterations = 0; info->rel_residual = 0.0; }
    return HB_OK;
  }
  hipLaunchKernelGGL(k_scale_copy, dim3(grid1d(n)), dim3(256), 0, s, b, 1.0 / beta, Q, n);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, dg, (size_t)1, beta);
  int it = 0;
  bool conv = false;
  auto converged = [&](int jj) { return c->h_res[jj] <= tol; };
  // the estimate after step jj + 1 extrapolated from steps jj - 1 and jj is within twice tol
  auto near_tol = [&](int jj) {
    const double r0 = c->h_res[jj - 1], r1 = c->h_res[jj];
    return r0 > 0.0 && r1 * (r1 / r0) <= 2.0 * tol;
  };
  for (int j = 0; j < m; ++j) {
    double *wj = Q + (size_t)(j + 1) * n;
    if (precond) {
      if ((rc = pc_apply(c, precond, Q + (size_t)j * n, r, s))) return rc;
      if ((rc = apply_V(c, op, r, wj, s))) return rc;
    } else if ((rc = apply_V(c, op, Q + (size_t)j * n, wj, s))) {
      return rc;
    }
    const size_t shm = sizeof(double) * (j + 1);
    hipLaunchKernelGGL(k_multi_dot, dim3(nchunk, j + 1), dim3(256), 0, s, Q, n, wj, n, p1, nchunk);
    hipLaunchKernelGGL(k_cgs_sub, dim3(nblk), dim3(256), shm, s, Q, n, p1, nchunk, j + 1, wj, n,
                       (double *)nullptr);
    hipLaunchKernelGGL(k_multi_dot, dim3(nchunk, j + 1), dim3(256), 0, s, Q, n, wj, n, p2, nchunk);
    hipLaunchKernelGGL(k_cgs_sub, dim3(nblk), dim3(256), shm, s, Q, n, p2, nchunk, j + 1, wj, n, pn);
    hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(256), sizeof(double) * 3 * (j + 1), s, dH, m, j, p1,
                       p2, nchunk, pn, nblk, dcs, dsn, dg, beta, dinv, res_dev);
    hipLaunchKernelGGL(k_scale_dev, dim3(grid1d(n)), dim3(256), 0, s, wj, dinv, n);
    HB_CHECK(c, hipGetLastError());
    HB_CHECK(c, hipEventRecord(c->ev_step, s));
    // step j is queued; look at step j - 1 (finished or about to) while it runs
    if (j > 0) {
      HB_CHECK(c, hipEventSynchronize(c->ev_prev));
      if (converged(j - 1)) {
        it = j;
        conv = true;
        break;
      }
      // step j may be the last: wait for it before queueing another one, which would otherwise
      // be computed for nothing
      if (j >= 2 && near_tol(j - 1)) {
        HB_CHECK(c, hipEventSynchronize(c->ev_step));
        if (converged(j)) {
          it = j + 1;
          conv = true;
          break;
        }
      }
    }
    std::swap(c->ev_step, c->ev_prev);
    it = j + 1;
  }
  if (!conv) {
    HB_CHECK(c, hipStreamSynchronize(s));
    conv = it > 0 && converged(it - 1);
  }
  // y = R^{-1} g over the first it columns, x = (P) Q y
  double *coef = dres;  // no longer needed
  std::vector<double> y;
  if (it > kBacksubMax) {
    std::vector<double> R((size_t)it * m), gh(it);
    y.resize(it);
    HB_CHECK(c, hipStreamSynchronize(s));
    HB_CHECK(c, hipMemcpy(R.data(), dH, sizeof(double) * (size_t)it * m, hipMemcpyDeviceToHost));
    HB_CHECK(c, hipMemcpy(gh.data(), dg, sizeof(double) * it, hipMemcpyDeviceToHost));
    for (int i = it - 1; i >= 0; --i) {
      double sacc = gh[i];
      for (int k = i + 1; k < it; ++k) sacc -= R[(size_t)i * m + k] * y[k];
      y[i] = sacc / R[(size_t)i * m + i];
    }
    HB_CHECK(c, hipMemcpyAsync(coef, y.data(), sizeof(double) * it, hipMemcpyHostToDevice, s));
  } else if (it > 0) {
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(256), sizeof(double) * ((size_t)it * it + 2 * it), s,
                       dH, m, dg, it, coef);
  }
  if (precond) {
    hipLaunchKernelGGL(k_combine, dim3(grid1d(n)), dim3(256), 0, s, Q, n, coef, it, r, n);
    if ((rc = pc_apply(c, precond, r, x, s))) return rc;
  } else {
    hipLaunchKernelGGL(k_combine, dim3(grid1d(n)), dim3(256), 0, s, Q, n, coef, it, x, n);
  }
  HB_CHECK(c, hipGetLastError());
  if (!y.empty()) HB_CHECK(c, hipStreamSynchronize(s));  // the host copy of y is read until here
  if (info) info->iterations = it;
  return conv ? HB_OK : HB_ENOCONV;
}

// Time marching (Sec. 3: the block lower-triangular system solved step by step): w^k = (V^0)^{-1}
// (b^k - sum_{d>=1} V^d w^{k-d}).  The steps [k0, k1) are split in halves: the first half is
// solved, one windowed Toeplitz product subtracts its contribution from the second half's right
// sides (blocks d = 1 .. k1 - k0 - 1, sources [k0, km), targets [km, k1)), then the second half is
// solved.  Runs of at most kTmLeaf steps go step by step, their own history subtracted block by
// block.  Every level of the halving reads each block about once, so the blocks are streamed
// about log2(E_t / kTmLeaf) + kTmLeaf / 2 + 1 times in all instead of E_t / 2 times; each product
// sees only its window of n steps, so its MFMA work covers n, not E_t, output times.
constexpr int kTmLeaf = 4;

static int tm_solve(hb_ctx *c, double *r, double *w, int k0, int k1, hipStream_t s) {
  const int ne = (int)c->ne;
  const size_t blk = (size_t)ne * ne;
  int rc;
  if (k1 - k0 <= kTmLeaf) {
    const void *V1 = (const char *)c->d_V + blk * (c->storage_f32 ? 4 : 8);
    for (int k = k0; k < k1; ++k) {
      // w^k = (V^0)^{-1} r^k
      if ((rc = gemv_batch(c, c->d_v0inv, 0, ne, ne, 1, r + (size_t)k * ne, w + (size_t)k * ne,
                           1.0, 0.0, 0, s)))
        return rc;
      // r^{k+d} -= V^d w^k inside the run, d = 1 .. k1-1-k
      if ((rc = gemv_batch(c, V1, blk, ne, ne, k1 - 1 - k, w + (size_t)k * ne,
                           r + (size_t)(k + 1) * ne, -1.0, 1.0, (size_t)ne, s)))
        return rc;
    }
    return HB_OK;
  }
  const int km = k0 + (k1 - k0) / 2, n = k1 - k0, h = km - k0;
  if ((rc = tm_solve(c, r, w, k0, km, s))) return rc;
  // the window [k0, k1): sources [0, h), targets [h, n)
  double *wv = w + (size_t)k0 * ne, *rv = r + (size_t)k0 * ne;
  if (c->storage_f32)
    rc = launch_toeplitz<float>(c, (const float *)c->d_V, ne, ne, wv, rv, s, 1, n, 0, h, true, h,
                                nullptr, 0, n, n);
  else
    rc = launch_toeplitz<double>(c, (const double *)c->d_V, ne, ne, wv, rv, s, 1, n, 0, h, true, h,
                                 nullptr, 0, n, n);
  if (rc) return rc;
  return tm_solve(c, r, w, km, k1, s);
}

int time_march(hb_ctx *c, const double *b, double *w, hipStream_t s) {
  const int nt = c->nt, ne = (int)c->ne;
  const size_t n = (size_t)nt * ne;
  int rc = invert_v0(c, s);
  if (rc) return rc;
  if ((rc = ensure_work(c, sizeof(double) * n))) return rc;
  double *r = c->d_work;
  HB_CHECK(c, hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (c->nu) {
    // non-uniform grid: w^k = (V^{k,k})^{-1} (b^k - sum_{i<k} V^{k,i} w^i), step by step
    const size_t nn = (size_t)ne * ne;
    for (int k = 0; k < nt; ++k) {
      if (k > 0) {
        hipLaunchKernelGGL(k_nu_hist, dim3((unsigned)((ne + 3) / 4)), dim3(256), 0, s,
                           (const double *)c->d_V, (const double *)w, r, k, ne, ne);
        HB_CHECK(c, hipGetLastError());
      }
      if ((rc = gemv_batch(c, c->d_v0inv + k * nn, 0, ne, ne, 1, r + (size_t)k * ne,
                           w + (size_t)k * ne, 1.0, 0.0, 0, s)))
        return rc;
    }
    return HB_OK;
  }
  return tm_solve(c, r, w, 0, nt, s);
}

// Two vectors of n doubles behind c->d_ir (residual and correction), shared with mixed_ir
int ensure_ir(hb_ctx *c, size_t n) {
  const size_t need = 2 * n * sizeof(double) + 64 * sizeof(double);
  if (c->ir_bytes >= need) return HB_OK;
  if (c->d_ir) (void)hipFree(c->d_ir);
  c->d_ir = nullptr;
  c->ir_bytes = 0;
  HB_CHECK(c, hipMalloc(&c->d_ir, need));
  c->ir_bytes = need;
  return HB_OK;
}

// Iterative refinement: x_{i+1} = x_i + d_i with V32 d_i ~= b - V_h x_i (GMRES on the float
// operator to relative tolerance inner_tol, at most maxit iterations each and `budget` in all);
// residuals in double with the double operator.
int mixed_ir(hb_ctx *c, const double *b, double *x, double tol, int maxit, int budget,
             hipStream_t s, hb_solve_info *info, bool precond) {
  const size_t n = (size_t)c->nt * c->ne;
  int rc = ensure_V32(c, s);
  if (rc) return rc;
  if ((rc = ensure_ir(c, n))) return rc;
  double *r = c->d_ir, *dlt = r + n;
  const double inner_tol = 1e-4;
  hipLaunchKernelGGL(k_fill, dim3(grid1d(n)), dim3(256), 0, s, x, n, 0.0);
  HB_CHECK(c, hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // norms via the GMRES dot kernels (scratch behind the correction vector is not needed)
  auto norm = [&](const double *v, double *out) -> int {
    const int nchunk = (int)((n + kDotChunk - 1) / kDotChunk);
    if (c->work_bytes < sizeof(double) * (nchunk + 2)) {
      int r2 = ensure_work(c, sizeof(double) * (nchunk + 2));
      if (r2) return r2;
    }
    double *partial = c->d_work, *dres = partial + nchunk;
    int r2 = multi_dot(c, v, 0, 1, v, n, partial, dres, out, s);
    *out = std::sqrt(*out);
    return r2;
  };
  double bn;
  if ((rc = norm(b, &bn))) return rc;
  if (bn == 0.0) return HB_OK;
  int total_it = 0, outer = 0;
  bool conv = false;
  for (; outer < 12; ++outer) {
    if (outer > 0) {
      if ((rc = apply_V(c, 0, x, r, s))) return rc;
      hipLaunchKernelGGL(k_axpby, dim3(grid1d(n)), dim3(256), 0, s, 1.0, b, -1.0, r, n);
    }
    double rn = bn;  // r = b while x = 0
    if (outer > 0 && (rc = norm(r, &rn))) return rc;
    if (rn <= tol * bn) {
      conv = true;
      break;
    }
    if (total_it >= budget) break;
    hb_solve_info in{};
    rc = gmres(c, 1, r, dlt, inner_tol, std::min(maxit, budget - total_it), s, &in, precond, rn);
    if (rc != HB_OK && rc != HB_ENOCONV) return rc;
    total_it += in.iterations;
    hipLaunchKernelGGL(k_axpby, dim3(grid1d(n)), dim3(256), 0, s, 1.0, dlt, 1.0, x, n);
  }
  if (info) {
    info->iterations = total_it;
    info->refinements = outer;
  }
  return conv ? HB_OK : HB_ENOCONV;
}

// r = b - A w with the double operator (op 0: V_h, 2: D_h) into r; *rn = ||r||, *bn = ||b||
int residual_norms(hb_ctx *c, int op, const double *b, const double *w, double *r, double *rn,
                   double *bn, hipStream_t s) {
  const size_t n = (size_t)c->nt * (op == 2 ? c->nv : c->ne);
  const int nchunk = (int)((n + kDotChunk - 1) / kDotChunk);
  int rc = ensure_work(c, sizeof(double) * (nchunk + 2));
  if (rc) return rc;
  double *partial = c->d_work, *dres = partial + nchunk;
  if ((rc = apply_V(c, op == 2 ? 2 : 0, w, r, s))) return rc;
  hipLaunchKernelGGL(k_axpby, dim3(grid1d(n)), dim3(256), 0, s, 1.0, b, -1.0, r, n);
  HB_CHECK(c, hipGetLastError());
  double rr, bb;
  if ((rc = multi_dot(c, r, 0, 1, r, n, partial, dres, &rr, s))) return rc;
  if ((rc = multi_dot(c, b, 0, 1, b, n, partial, dres, &bb, s))) return rc;
  *rn = std::sqrt(rr);
  *bn = std::sqrt(bb);
  return HB_OK;
}

// The residual contract of hb_solve / hb_solve_neumann (Sec. 6.1: the relative residual in the
// double operator decides).  After the chosen method has produced w (rc0 its status), the
// residual r = b - A w is recomputed in double; while ||r|| > tol ||b|| the solve continues from
// w: GMRES on A delta = r to the tolerance that brings b - A (w + delta) below half the target,
// w += delta (a restart), within the iteration budget; time marching repeats its exact forward
// substitution on r (at most three times).  A preconditioned or mixed-precision phase that ended
// without reaching the target hands over to plain double GMRES (the fallback), which also
// carries every later restart.  HB_OK only if ||b - A w|| <= tol ||b|| at the end.
// op: 0 V_h (pc_kind 1: the learned map), 2 D_h (pc_kind 2: the operator preconditioner).
int enforce_residual(hb_ctx *c, int op, int method, int pc_kind, const double *b, double *w,
                     const hb_solve_opts &o, int rc0, hb_solve_info &inf, hipStream_t s) {
  const size_t n = (size_t)c->nt * (op == 2 ? c->nv : c->ne);
  int rc = ensure_ir(c, n);
  if (rc) return rc;
  double *r = c->d_ir, *dlt = r + n;
  double rn = 0.0, bn = 0.0;
  if ((rc = residual_norms(c, op, b, w, r, &rn, &bn, s))) return rc;
  const bool timemarch = method == HB_SOLVE_TIMEMARCH;
  // the phase that produced w did not reach its target: plain double GMRES from here on
  bool plain = rc0 == HB_ENOCONV && (pc_kind != 0 || method == HB_SOLVE_MIXED_IR);
  if (plain) inf.fallback = 1;
  // iterations left: mixed refinement counts max_iter per inner solve, so its fallback starts
  // with a full budget; GMRES shares one budget over all phases
  int used = method == HB_SOLVE_MIXED_IR ? 0 : inf.iterations;
  while (bn > 0.0 && rn > o.tol * bn) {
    if (timemarch) {
      if (inf.restarts >= 3) break;
      if ((rc = time_march(c, r, dlt, s))) return rc;
    } else {
      const int left = o.max_iter - used;
      if (left <= 0) break;
      hb_solve_info ii{};
      const int kind = plain ? 0 : pc_kind;
      rc = gmres(c, op, r, dlt, 0.5 * o.tol * bn / rn, left, s, &ii, kind, rn);
      if (rc != HB_OK && rc != HB_ENOCONV) return rc;
      used += ii.iterations;
      inf.iterations += ii.iterations;
      if (rc == HB_ENOCONV && kind != 0) {
        plain = true;
        inf.fallback = 1;
      }
    }
    hipLaunchKernelGGL(k_axpby, dim3(grid1d(n)), dim3(256), 0, s, 1.0, dlt, 1.0, w, n);
    HB_CHECK(c, hipGetLastError());
    inf.restarts += 1;
    if ((rc = residual_norms(c, op, b, w, r, &rn, &bn, s))) return rc;
  }
  inf.rel_residual = bn > 0.0 ? rn / bn : 0.0;
  return bn == 0.0 || rn <= o.tol * bn ? HB_OK : HB_ENOCONV;
}

}  // namespace

extern "C" {

// K_h^T: the transposed blocks are formed once per assembly of K
static int ensure_Kt(hb_ctx *c, hipStream_t s) {
  if (c->Kt_valid) return HB_OK;
  const size_t bytes = (size_t)c->nt * c->ne * c->nv * (c->storage_f32 ? 4 : 8);
  if (!c->d_Kt) {
    HB_CHECK(c, hipMalloc(&c->d_Kt, bytes + kBlockPad));
    HB_CHECK(c, hipMemsetAsync((char *)c->d_Kt + bytes, 0, kBlockPad, s));
  }
  int rc = launch_transpose_blocks(c, c->d_K, c->d_Kt, (int)c->ne, (int)c->nv, s);
  if (rc) return ctx_fail(c, rc, "block transpose launch failed");
  c->Kt_valid = true;
  return HB_OK;
}

int hb_apply(hb_ctx *c, uint32_t op, const double *x, double *y, void *stream) {
  if (!c) return HB_EINVAL;
  if (!x || !y) return ctx_fail(c, HB_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  if (c->nu) {
    if (op != HB_OP_V && op != HB_OP_K)
      return ctx_fail(c, HB_EINVAL, "a non-uniform grid has HB_OP_V and HB_OP_K only");
    if (op == HB_OP_V ? !c->have_V : !c->have_K) return ctx_fail(c, HB_ESTATE, "operator not assembled");
    return nu_apply(c, (const double *)(op == HB_OP_V ? c->d_V : c->d_K), (int)c->ne,
                    (int)(op == HB_OP_V ? c->ne : c->nv), x, y, s);
  }
  if (op == HB_OP_D || op == HB_OP_V11) {
    if (op == HB_OP_D ? !c->have_D : !c->have_V11) return ctx_fail(c, HB_ESTATE, "operator not assembled");
    return toeplitz_apply(c, op == HB_OP_D ? c->d_D : c->d_V11, (int)c->nv, (int)c->nv, x, y, s);
  }
  if (op == HB_OP_KT) {
    if (!c->have_K) return ctx_fail(c, HB_ESTATE, "operator not assembled");
    int rc = ensure_Kt(c, s);
    if (rc) return rc;
    return toeplitz_apply(c, c->d_Kt, (int)c->nv, (int)c->ne, x, y, s);
  }
  if (op != HB_OP_V && op != HB_OP_K)
    return ctx_fail(c, HB_EINVAL, "op must be HB_OP_V, HB_OP_K, HB_OP_D, HB_OP_V11 or HB_OP_KT");
  if (op == HB_OP_V ? !c->have_V : !c->have_K) return ctx_fail(c, HB_ESTATE, "operator not assembled");
  return toeplitz_apply(c, op == HB_OP_V ? c->d_V : c->d_K, (int)c->ne,
                        (int)(op == HB_OP_V ? c->ne : c->nv), x, y, s);
}

int hb_apply_noalloc(hb_ctx *c, uint32_t op, const double *x, double *y, void *stream) {
  if (!c) return HB_EINVAL;
  if (!x || !y) return ctx_fail(c, HB_EINVAL, "null vector");
  if (c->nu) return ctx_fail(c, HB_EINVAL, "not available on a non-uniform time grid (hb_apply allocates nothing there)");
  hipStream_t s = (hipStream_t)stream;
  void *P = static_scratch(c);
  if (!P) return ctx_fail(c, HB_ESTATE, "fixed scratch not set up on this context's device");
  const size_t rows = (op == HB_OP_V || op == HB_OP_K) ? (size_t)c->ne : (size_t)c->nv;
  if ((size_t)c->nt * rows * (c->storage_f32 ? sizeof(float) : sizeof(double)) > kStaticScratchBytes)
    return ctx_fail(c, HB_EINVAL, "E_t x rows x element size exceeds the 32 MiB fixed scratch");
  const void *blocks;
  int R, C;
  if (op == HB_OP_V || op == HB_OP_K) {
    if (op == HB_OP_V ? !c->have_V : !c->have_K) return ctx_fail(c, HB_ESTATE, "operator not assembled");
    blocks = op == HB_OP_V ? c->d_V : c->d_K;
    R = (int)c->ne;
    C = (int)(op == HB_OP_V ? c->ne : c->nv);
  } else if (op == HB_OP_D || op == HB_OP_V11) {
    if (op == HB_OP_D ? !c->have_D : !c->have_V11) return ctx_fail(c, HB_ESTATE, "operator not assembled");
    blocks = op == HB_OP_D ? c->d_D : c->d_V11;
    R = C = (int)c->nv;
  } else if (op == HB_OP_KT) {
    if (!c->have_K) return ctx_fail(c, HB_ESTATE, "operator not assembled");
    // the transposed blocks need a buffer of their own: only an hb_apply(HB_OP_KT) made after
    // the last assembly of K has formed them
    if (!c->Kt_valid) return ctx_fail(c, HB_ESTATE, "K_h^T not formed since the last assembly of K (call hb_apply with HB_OP_KT once)");
    blocks = c->d_Kt;
    R = (int)c->nv;
    C = (int)c->ne;
  } else {
    return ctx_fail(c, HB_EINVAL, "op must be HB_OP_V, HB_OP_K, HB_OP_D, HB_OP_V11 or HB_OP_KT");
  }
  const int nt = c->nt;
  if (c->storage_f32)
    return launch_toeplitz<float>(c, (const float *)blocks, R, C, x, y, s, 0, nt, 0, nt, false, 0,
                                  P, kStaticScratchBytes);
  return launch_toeplitz<double>(c, (const double *)blocks, R, C, x, y, s, 0, nt, 0, nt, false, 0,
                                 P, kStaticScratchBytes);
}

int hb_rhs_neumann(hb_ctx *c, const double *psi, double *b, void *stream) {
  if (!c) return HB_EINVAL;
  if (!psi || !b) return ctx_fail(c, HB_EINVAL, "null vector");
  if (c->nu) return ctx_fail(c, HB_EINVAL, "not available on a non-uniform time grid");
  if (!c->have_K) return ctx_fail(c, HB_ESTATE, "K not assembled");
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_Kt(c, s);
  if (rc) return rc;
  if ((rc = toeplitz_apply(c, c->d_Kt, (int)c->nv, (int)c->ne, psi, b, s))) return rc;
  const size_t n = (size_t)c->nt * c->nv;
  hipLaunchKernelGGL(k_mass_half_T, dim3(grid1d(n)), dim3(256), 0, s, c->d_mass, c->d_vstart,
                     c->d_vadj, psi, b, c->nt, (int)c->ne, (int)c->nv, 0.5 * c->h);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

int hb_solve_neumann(hb_ctx *c, const double *b, double *u, const hb_solve_opts *opts,
                     hb_solve_info *info, void *stream) {
  if (!c) return HB_EINVAL;
  if (!b || !u) return ctx_fail(c, HB_EINVAL, "null vector");
  if (c->nu) return ctx_fail(c, HB_EINVAL, "not available on a non-uniform time grid");
  if (!c->have_D) return ctx_fail(c, HB_ESTATE, "D not assembled");
  hb_solve_opts o{};
  o.method = HB_SOLVE_GMRES;
  o.max_iter = 500;
  o.tol = 1e-8;
  if (opts) {
    o = *opts;
    if (o.max_iter <= 0) o.max_iter = 500;
    if (!(o.tol > 0)) o.tol = 1e-8;
  }
  if (o.method != HB_SOLVE_GMRES)
    return ctx_fail(c, HB_EINVAL, "the Neumann system is solved by GMRES only");
  if (o.precond != 0 && o.precond != 1) return ctx_fail(c, HB_EINVAL, "precond must be 0 or 1");
  if (o.precond && !c->have_V11) return ctx_fail(c, HB_ESTATE, "the preconditioner needs HB_OP_V11");
  if (o.max_iter > 5000) return ctx_fail(c, HB_EINVAL, "max_iter must be <= 5000");
  hipStream_t s = (hipStream_t)stream;
  hb_solve_info inf{};
  HB_CHECK(c, hipStreamSynchronize(s));
  auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (o.precond && (rc = ensure_minv(c, s))) return rc;
  const int cap = o.precond && o.precond_max_iter > 0 ? std::min(o.precond_max_iter, o.max_iter)
                                                      : o.max_iter;
  rc = gmres(c, 2, b, u, o.tol, cap, s, &inf, o.precond ? 2 : 0);
  if (rc != HB_OK && rc != HB_ENOCONV) return rc;
  rc = enforce_residual(c, 2, HB_SOLVE_GMRES, o.precond ? 2 : 0, b, u, o, rc, inf, s);
  if (rc != HB_OK && rc != HB_ENOCONV) return rc;
  HB_CHECK(c, hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  inf.seconds = std::chrono::duration<double>(t1 - t0).count();
  if (info) *info = inf;
  if (rc == HB_ENOCONV) c->err = "the relative residual is above tol after max_iter iterations";
  return rc;
}

int hb_rhs_dirichlet(hb_ctx *c, const double *g, double *b, void *stream) {
  if (!c) return HB_EINVAL;
  if (!g || !b) return ctx_fail(c, HB_EINVAL, "null vector");
  if (!c->have_K) return ctx_fail(c, HB_ESTATE, "K not assembled");
  hipStream_t s = (hipStream_t)stream;
  if (c->nu) {
    int rc = nu_apply(c, (const double *)c->d_K, (int)c->ne, (int)c->nv, g, b, s);
    if (rc) return rc;
    const size_t n = (size_t)c->nt * c->ne;
    hipLaunchKernelGGL(k_mass_half_steps, dim3(grid1d(n)), dim3(256), 0, s, c->d_mass, c->d_tris, g,
                       b, c->nt, (int)c->ne, (int)c->nv, c->d_nu_h);
    HB_CHECK(c, hipGetLastError());
    return HB_OK;
  }
  int rc = toeplitz_apply(c, c->d_K, (int)c->ne, (int)c->nv, g, b, s);
  if (rc) return rc;
  const size_t n = (size_t)c->nt * c->ne;
  hipLaunchKernelGGL(k_mass_half, dim3(grid1d(n)), dim3(256), 0, s, c->d_mass, c->d_tris, g, b,
                     c->nt, (int)c->ne, (int)c->nv, 0.5 * c->h);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

int hb_solve(hb_ctx *c, const double *b, double *w, const hb_solve_opts *opts, hb_solve_info *info,
             void *stream) {
  if (!c) return HB_EINVAL;
  if (!b || !w) return ctx_fail(c, HB_EINVAL, "null vector");
  if (!c->have_V) return ctx_fail(c, HB_ESTATE, "V not assembled");
  hb_solve_opts o{};
  o.method = HB_SOLVE_GMRES;
  o.max_iter = 500;
  o.tol = 1e-8;
  if (opts) {
    o = *opts;
    if (o.max_iter <= 0) o.max_iter = 500;
    if (!(o.tol > 0)) o.tol = 1e-8;
  }
  if (o.method != HB_SOLVE_GMRES && o.method != HB_SOLVE_TIMEMARCH && o.method != HB_SOLVE_MIXED_IR)
    return ctx_fail(c, HB_EINVAL, "unknown solver method");
  if (c->nu && (o.method == HB_SOLVE_MIXED_IR || o.precond))
    return ctx_fail(c, HB_EINVAL,
                    "a non-uniform grid is solved by GMRES or time marching without preconditioner");
  if (o.max_iter > 5000) return ctx_fail(c, HB_EINVAL, "max_iter must be <= 5000");
  hipStream_t s = (hipStream_t)stream;
  hb_solve_info inf{};
  // the solve blocks anyway (GMRES reads its residual estimates); work queued before it on the
  // stream is drained first so that it does not count as solve time
  HB_CHECK(c, hipStreamSynchronize(s));
  auto t0 = std::chrono::steady_clock::now();
  int rc;
  if (o.precond && !c->pc_active) return ctx_fail(c, HB_ESTATE, "no preconditioner installed");
  const bool pc = o.precond != 0;
  const int cap = pc && o.precond_max_iter > 0 ? std::min(o.precond_max_iter, o.max_iter)
                                               : o.max_iter;
  if (o.method == HB_SOLVE_GMRES) rc = gmres(c, 0, b, w, o.tol, cap, s, &inf, pc);
  else if (o.method == HB_SOLVE_MIXED_IR)
    rc = mixed_ir(c, b, w, o.tol, o.max_iter, o.precond_max_iter > 0 ? o.precond_max_iter : INT32_MAX,
                  s, &inf, pc);
  else rc = time_march(c, b, w, s);
  if (rc != HB_OK && rc != HB_ENOCONV) return rc;
  rc = enforce_residual(c, 0, o.method, pc ? 1 : 0, b, w, o, rc, inf, s);
  if (rc != HB_OK && rc != HB_ENOCONV) return rc;
  HB_CHECK(c, hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  inf.seconds = std::chrono::duration<double>(t1 - t0).count();
  if (info) *info = inf;
  if (rc == HB_ENOCONV) c->err = "the relative residual is above tol after max_iter iterations";
  return rc;
}

int hb_eval_repr(hb_ctx *c, const double *pts, int64_t P, const double *w, const double *g,
                 double *u, double *sl, double *dl, void *stream) {
  if (!c) return HB_EINVAL;
  if (P < 0) return ctx_fail(c, HB_EINVAL, "P must be >= 0");
  if (P == 0) return HB_OK;
  if (!pts || !w || !g || !u) return ctx_fail(c, HB_EINVAL, "null pointer");
  if (P > (int64_t)1 << 31) return ctx_fail(c, HB_EINVAL, "too many points");
  hipStream_t s = (hipStream_t)stream;
  if (!c->d_params_repr) {
    HB_CHECK(c, hipMalloc(&c->d_params_repr, sizeof(AsmParams)));
    HB_CHECK(c, hipMemcpy(c->d_params_repr, &c->params, sizeof(AsmParams), hipMemcpyHostToDevice));
  }
  if (c->nu) {
    const size_t lds = sizeof(double) * ((size_t)c->nt + 1);
    if (lds + sizeof(double) * 8 > 160 * 1024)
      return ctx_fail(c, HB_EINVAL, "E_t too large for the potential kernel");
    hipLaunchKernelGGL(k_nu_repr, dim3((unsigned)P), dim3(256), lds, s, c->d_params_repr,
                       c->d_nu_t, pts, w, g, u, sl, dl);
    HB_CHECK(c, hipGetLastError());
    return HB_OK;
  }
  if (!c->d_reprq) {
    // Q_{2k}(w) / (2k+1)! for p = 3/2 (Q_0 = 1, Q_{n+1} = (w - n - p) Q_n - w Q_n'), the building
    // blocks of the interval averages of the potentials' time integrals (the double layer's
    // series follows from these by S_{5/2} = S_{3/2} - S_{3/2}')
    std::vector<double> q(kReprQ * (kReprDeg + 1), 0.0);
    {
      const long double pw = 1.5L;
      std::vector<long double> cur(1, 1.0L);
      long double fact = 1.0L;  // (n+1)! for n = 0
      for (int n = 0; n <= kReprDeg; ++n) {
        if (n > 0) fact *= (long double)(n + 1);
        if (n % 2 == 0)
          for (size_t jj = 0; jj < cur.size(); ++jj)
            q[(size_t)(n / 2) * (kReprDeg + 1) + jj] = (double)(cur[jj] / fact);
        std::vector<long double> nx(cur.size() + 1, 0.0L);
        for (size_t jj = 0; jj < cur.size(); ++jj) {
          nx[jj + 1] += cur[jj];
          nx[jj] -= ((long double)n + pw + (long double)jj) * cur[jj];
        }
        cur.swap(nx);
      }
    }
    HB_CHECK(c, hipMalloc(&c->d_reprq, q.size() * sizeof(double)));
    HB_CHECK(c, hipMemcpy(c->d_reprq, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  // per-interval coefficient tables of the largest interval count
  int moff = 0;
  {
    const int lo[6] = {3, 4, 6, 8, 16, 32}, hi[6] = {4, 6, 8, 16, 32, 1 << 30};
    const int deg[6] = {20, 16, 14, 12, 10, 8};
    for (int cl = 0; cl < 6; ++cl)
      moff += std::max(0, std::min(c->nt + 1, hi[cl]) - lo[cl]) * (3 + deg[cl] + 1);
  }
  const size_t lds = std::max<size_t>(8, sizeof(double) * (size_t)moff);
  // 160 KiB of LDS per workgroup, less the kernel's static arrays (Q, the exp table, the reduction)
  if (lds + sizeof(double) * (kReprQ * (kReprDeg + 1) + kExpTabN + 8) > 160 * 1024)
    return ctx_fail(c, HB_EINVAL, "E_t too large for the potential kernel");
  hipLaunchKernelGGL(k_repr, dim3((unsigned)P), dim3(256), lds, s, c->d_params_repr, c->d_reprq,
                     pts, w, g, u, sl, dl);
  HB_CHECK(c, hipGetLastError());
  return HB_OK;
}

}  // extern "C"
