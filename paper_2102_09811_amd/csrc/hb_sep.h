// Device helpers of the pair kernels (V_h / K_h and the p1 x p1 blocks): the wave's test-panel
// rule nodes in LDS, the per-task table of distinct trial vertices, and a DPP lane move.
#pragma once
#include "hb_device.h"
#include "hb_internal.h"

namespace hb {

struct RuleNode {
  double x, y, z, w;
};
__device__ __forceinline__ RuleNode rule_node(const double *q, int a) {
  const double2 u = *(const double2 *)(q + 4 * a), v = *(const double2 *)(q + 4 * a + 2);
  return {u.x, u.y, v.x, v.y};
}

// LDS staging of the separated kernels (before any lane leaves): the workgroup's barycentric
// table, and each wave's test-panel nodes (lanes 0 .. 20 of the wave).
__device__ __forceinline__ void stage_test_nodes(const AsmParams &p, const double *geom, int l,
                                                 bool valid, double *xs_wave, double *lam) {
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < kFarN * 4) {
    const int a = threadIdx.x >> 2, c = threadIdx.x & 3;
    lam[threadIdx.x] = c < 3 ? p.lam7[a][c] : p.w7[a];
  }
  if (valid && lane < kFarN * 4) {
    const int a = lane >> 2, c = lane & 3;
    xs_wave[lane] = c < 3 ? geom[(size_t)(a * 3 + c) * p.ne + l] : p.w7[a];
  }
}

// LDS of the wave, ordered: earlier LDS operations of any lane are seen by later ones.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kSepSlots = 3 * 64;  // distinct trial vertices of one task, at most

// The 11 columns of a regularised rule table (SoA [11][n]) as uniform base pointers: a lane reads
// entry q of column k at base k + 8 q bytes, one 32-bit offset for all columns, so the loads need
// no per-column address arithmetic.
struct RuleCols {
  const char *c[11];
  RuleCols() = default;
  __device__ RuleCols(const double *tab, int n) {
#pragma unroll
    for (int k = 0; k < 11; ++k) c[k] = (const char *)(tab + (size_t)k * n);
  }
  __device__ __forceinline__ double at(int k, unsigned off) const {
    return *(const double *)(c[k] + off);
  }
};

// v from the lane given by the DPP control CTRL within each row of sixteen lanes
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

}  // namespace hb
