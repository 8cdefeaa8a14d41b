// Internal declarations shared by the host runtime (hb_host.cpp) and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/heatbem.h"

struct hb_ctx;

namespace hb {

// Blocks 0 .. d_switch-1 come from second differences of G^{dtau dt} at the closed-form levels
// 0 .. d_switch; later blocks use the Taylor form, whose degree falls as d grows (28 at d = 3).
constexpr int kTaylorDeg = 28;       // largest degree of the Taylor polynomial in w = rho^2/(4 alpha d h)
constexpr int kTaylorN = kTaylorDeg + 1;
// Polynomial lengths the double-precision Taylor passes of k_separated and k_touching are
// instantiated for (ascending; the host rounds a pass's length up to one of them).
constexpr int kPolyLens[] = {5, 6, 7, 8, 9, 10, 11, 13, 15, 17, 19, 21, 25, 29};
// The same for the odd polynomials of D^{2,d} in the hypersingular kernels.
constexpr int kD2Lens[] = {4, 6, 8, 10, 12, 14, 16, 20, 24};
constexpr int kTaylorDeg32 = 16;     // largest degree of the float evaluation (mixed precision)
constexpr int kTaylorN32 = kTaylorDeg32 + 1;
constexpr int kSeriesN = 14;         // terms of the small-z series of the brackets A(z), B(z)
constexpr int kMaxClosed = 16;       // largest supported d_switch
constexpr int kFarN = 7;             // Radon 7-point rule
constexpr int kReprDeg = 20;         // largest degree of the potentials' Taylor polynomials
constexpr int kReprQ = kReprDeg / 2 + 1;
// Zeroed bytes behind every block array read by the Toeplitz product (V, K and the float copy of
// V): its fragment loads may run up to one column chunk less one entry past the last row of the
// last block (checked where the chunk width is defined).
constexpr size_t kBlockPad = 256;

// Per-level constants of the closed form at delta_i = i h (i = 0 .. d_switch).
struct LevelConsts {
  double c[kMaxClosed + 1];   // 1 / (2 sqrt(alpha delta_i))   (z = rho * c)
  double s2[kMaxClosed + 1];  // 2 alpha delta_i
  double s1[kMaxClosed + 1];  // 2 sqrt(alpha delta_i) / sqrt(pi)
  double t2[kMaxClosed + 1];  // 4 sqrt(alpha delta_i) / sqrt(pi)  (rho A(z) as rho -> 0)
};

struct AsmParams {
  int32_t ne, nv, nt, dsw;     // E_x, N_x, E_t, first Taylor block
  int32_t mixed_d_min;         // first d of float separated pairs (>= nt: none)
  double alpha, h;
  LevelConsts lv;
  double serA[kSeriesN];       // z * sum serA[n] z^{2n}  : part of sqrt(pi) A(z) - 2/z
  double serB[kSeriesN];       // z * sum serB[n] z^{2n}  : sqrt(pi)/4 B(z)
  double w7[kFarN];            // Radon weights (sum 1)
  double lam7[kFarN][3];       // Radon barycentric nodes
  // scale factors applied to the raw sums (see the kernels)
  double kV;                   // 1 / (8 pi alpha^2)
  double kVs;                  // h / (4 pi alpha)
  double kK;                   // 1 / (8 pi alpha)
  double kKs;                  // h / (4 pi)
  const double *taylor;        // [nt][2][kTaylorN] Taylor polynomials in w (V, K), d >= dsw
  const float *taylor32;       // [nt][2][kTaylorN32] shorter series for the float path
  const int32_t *tdeg;         // [nt][2]: polynomial degree of block d, double and float path
  const int32_t *tlen_sep;     // [nt]: polynomial length of the separated pairs' pass from block d
                               // (bounded by the mesh's extent)
  const int32_t *tlen_touch;   // [nt]: the same for the touching pairs (their distances are short,
                               // so the series in w is cut earlier)
  const double *tscale;        // [nt][3]: V scale, K scale, c_d = 1/(4 alpha d h)
  const double *geom;          // SoA [25][ne]: far nodes (q*3+c), normal (21..23), area (24)
  const int32_t *tris;         // [ne][3]
  void *V;                     // [nt][ne][ne]
  void *K;                     // [nt][ne][nv]
  void *KT;                    // [nt][nv][ne]: double-layer contributions of the transposed order
                               // of separated pairs, vertex-major so that a wave's atomics are
                               // contiguous; folded into K after the separated kernel
  int32_t do_V, do_K;
};

// One ordered touching pair (test l, trial m) with the vertex orders of the regularised rule.
struct TouchPair {
  int32_t l, m, cls, pad0;
  int32_t vtx[3], pad1;        // trial vertices in the rule's order (p1 basis lambda_k)
  double E1[3], E2[3];         // test panel edges  v1-v0, v2-v1 (rule order)
  double F1[3], F2[3];         // trial panel edges
  double n[3];                 // trial outward unit normal
  double scale;                // 4 * area_l * area_m
  int32_t vtxl[3], pad2;       // test vertices in the rule's order (hypersingular p1 x p1 blocks)
  double nn;                   // n_l . n_m
};

// Regularised rule of one class, SoA, padded to a multiple of 64 with zero weights.
struct SSRule {
  int32_t n = 0;               // padded count
  double *d = nullptr;         // device: [11][n] = c1, c2, c3, c4, w, lam0, lam1, lam2 (trial),
                               // lamx0, lamx1, lamx2 (test barycentrics, rule order)
};

// The three classes' rule tables as one kernel argument (index = shared vertices, 1..3).
struct RuleTabs {
  const double *d[4];
  int32_t n[4];
};

// ---- Non-uniform time steps (blocks V^{k,i}, K^{k,i}, 0 <= i <= k < E_t, of a graded grid) ----
// Block (k, i) is stored at index k (k + 1) / 2 + i.  Blocks whose gap t_k - t_{i+1} is small
// against their support are "closed" (the four-term difference of G^{dtau dt} per point); the
// others use the even Taylor series of the trapezoid-weighted kernel about the support's centre,
// with the tables laid out as the uniform Taylor tables (entry b of the Taylor list).
constexpr int kNuLev = 4;            // levels of a closed block
struct NuClosed {
  int32_t out;                       // packed block index
  int32_t diag;                      // 1: i = k (adds h_k G^{dtau}(rho, 0))
  int32_t nlev, pad;
  double c[kNuLev];                  // 1 / (2 sqrt(alpha delta)); 0 marks delta = 0 (the limit)
  double s2[kNuLev];                 // 2 alpha delta
  double s1[kNuLev];                 // 2 sqrt(alpha delta) / sqrt(pi)
  double t2[kNuLev];                 // 4 sqrt(alpha delta) / sqrt(pi)
  double sg[kNuLev];                 // +1 / -1
  double kVs, kKs;                   // h_k / (4 pi alpha), h_k / (4 pi) (diagonal blocks)
};
struct NuTabs {
  const NuClosed *closed;            // [n_closed]
  int32_t n_closed;
  int32_t n_taylor;                  // Taylor blocks, taken in pairs (b, b + 1)
  const int32_t *tout;               // [n_taylor]: packed block index of Taylor entry b
  const double *taylor;              // [n_taylor][2][kTaylorN]
  const double *tscale;              // [n_taylor][3]: V scale, K scale, 1 / (4 alpha c_b)
  const int32_t *tdeg;               // [n_taylor][2]: polynomial length of the pass (b, b + 1) that
                                     // entry b belongs to, separated and touching pairs (one of
                                     // kPolyLens: the pair's distance-bounded prefix)
};
void launch_nu_separated(const AsmParams *dp, const NuTabs &nu, const int32_t *tasks,
                         int64_t ntasks, hipStream_t s);
void launch_nu_touching(const AsmParams *dp, const NuTabs &nu, const TouchPair *pairs,
                        int64_t npairs, const SSRule rules[4], hipStream_t s);
// y^k = sum_{i <= k} A^{k,i} x^i over packed blocks [nb][R][C] (y overwritten, time-major)
int nu_apply(hb_ctx *c, const double *A, int R, int C, const double *x, double *y, hipStream_t s);

// dp: device copy of p (kernels read their parameters from device memory)
// tasks: (test panel, first trial panel, lanes) per wave; vstart / verts: each task's distinct
// trial vertices (CSR); slots: [task][3][64] the slot of each lane's trial vertex k
void launch_assemble_separated(const AsmParams *dp, const AsmParams &p, const int32_t *tasks,
                               const int32_t *vstart, const int32_t *verts, const uint8_t *slots,
                               int64_t ntasks, int precision, int storage_f32, hipStream_t s);
void launch_fold_KT(const AsmParams &p, int storage_f32, hipStream_t s);
// list: entries of the touching-pair kernels, pair indices, the last nsym of them ~index for
// pairs sharing one vertex that are integrated once for both orders (hb_ctx::d_touch_list)
void launch_assemble_touching(const AsmParams *dp, const AsmParams &p, const TouchPair *pairs,
                              const int32_t *list, int64_t nlist, int64_t nsym,
                              const SSRule rules[4], int storage_f32, hipStream_t s);

// Hypersingular operator (Sec. 3.3): D_h^d = D_h^{1,d} + D_h^{2,d} into c->d_D (needs V_h);
// Taylor form of D^{2,d} from block kD2Closed on, closed form below.
constexpr int kD2Closed = 4;
constexpr int kTaylorND = 24;        // coefficients of the odd Taylor polynomial of D^{2,d}, d >= 4
int launch_assemble_d(hb_ctx *c, hipStream_t s);
// V_h^{11}: the single layer between p1 test and trial functions (the paper's preconditioner
// matrix for D_h, Sec. 6.1) into c->d_V11, same rules and temporal forms as V_h
int launch_assemble_v11(hb_ctx *c, hipStream_t s);
// Near-field blocks of the listed ordered pairs (hb_nearfield_pattern): V[d][e], K[d][e][3]
int launch_assemble_near(hb_ctx *c, double *V, double *K, hipStream_t s);
// blockwise transpose [nt][R][C] -> [nt][C][R]
int launch_transpose_blocks(hb_ctx *c, const void *src, void *dst, int R, int C, hipStream_t s);

// Looks up this context's device copy of the fixed scratch of hb_apply_noalloc (once per device,
// with the device current); called by hb_create.
int static_scratch_init(hb_ctx *c);

// message of the last failed call made without a context (hb_last_error(NULL))
void set_global_error(const std::string &msg);

// y = A x for the block-Toeplitz operator with blocks [nt][R][C] (y overwritten, time-major)
int toeplitz_apply(hb_ctx *c, const void *blocks, int R, int C, const double *x, double *y,
                   hipStream_t s);
// z = diag(M, ..., M) q with the installed sparse approximate inverse
int precond_apply(hb_ctx *c, const double *q, double *z, hipStream_t s);
// same product with float blocks on the float MFMA path (float accumulation)
int toeplitz_apply32(hb_ctx *c, const float *blocks, int R, int C, const double *x, double *y,
                     hipStream_t s);

}  // namespace hb

struct hb_ctx {
  std::string err;
  int64_t ne = 0, nv = 0;
  int32_t nt = 0;
  double alpha = 0, T = 0, h = 0;
  hb_options opt{};
  std::vector<double> verts;
  std::vector<int32_t> tris;
  std::vector<double> area, normal;
  std::vector<hb::TouchPair> touch;  // sorted by class 3, 2, 1
  int64_t n_class[4] = {0, 0, 0, 0};
  int device = 0;
  // device data
  double *d_geom = nullptr;
  int32_t *d_tris = nullptr;
  hb::TouchPair *d_touch = nullptr;
  int32_t *d_touch_list = nullptr;   // entries of the touching-pair assembly (see the launcher)
  int64_t n_touch_list = 0, n_touch_sym = 0;
  int32_t *d_sep_tasks = nullptr;    // [n][3]: (test panel l, first trial panel m0, lanes) per wave;
                                     // lane i takes trial panel (m0 + i) mod E_x
  int64_t n_sep_tasks = 0;
  int32_t *d_sep_vstart = nullptr;   // [n_sep_tasks + 1]: CSR of the tasks' distinct trial vertices
  int32_t *d_sep_verts = nullptr;
  uint8_t *d_sep_slots = nullptr;    // [n_sep_tasks][3][64]: slot of each lane's trial vertex k
  hb::SSRule ss[4];
  double *d_taylor = nullptr, *d_tscale = nullptr;
  float *d_taylor32 = nullptr;
  int32_t *d_tdeg = nullptr, *d_tlen_sep = nullptr, *d_tlen_touch = nullptr;
  float *d_V32 = nullptr;            // float copy of V for the mixed-precision inner solver
  bool V32_valid = false;
  double *d_mass = nullptr;          // p0 x p1 mass, [ne][3] = area/3 per local vertex
  void *d_V = nullptr, *d_K = nullptr, *d_KT = nullptr;
  bool have_V = false, have_K = false;
  // hypersingular operator: blocks [nt][nv][nv], workspace of the separated pairs' half, tables
  void *d_D = nullptr, *d_Dw = nullptr;
  bool have_D = false;
  void *d_V11 = nullptr;             // [nt][nv][nv]: single layer between p1 functions
  bool have_V11 = false;
  double *d_minv = nullptr;          // inverse of the p1 mass matrix (+ elimination workspace)
  bool minv_valid = false;
  double *d_pcw = nullptr;           // operator preconditioner: two vectors of E_t x N_x
  size_t pcw_n = 0;
  // near-field pattern: ordered pairs (l, m) by rows; separated entries (l, m, entry) and
  // touching entries (touching-list index, entry, local trial vertex of rule vertex 0, 1, 2)
  int64_t near_nnz = -1, near_nsep = 0, near_ntouch = 0;
  std::vector<int64_t> near_start;
  std::vector<int32_t> near_cols;
  int32_t *d_near_sep = nullptr, *d_near_touch = nullptr;
  void *d_Kt = nullptr;              // K^d transposed block by block (K_h^T of the Neumann system)
  bool Kt_valid = false;
  double *d_d2tab = nullptr;         // [nt][kTaylorND]: odd Taylor polynomial of D^{2,d}
  double *d_d2scale = nullptr;       // [nt]: alpha h (4 pi alpha d h)^{-3/2}
  int32_t *d_d2len = nullptr;        // [nt][2]: coefficients used by the pass from block d,
                                     // separated and touching pairs (0 below kD2Closed)
  double *d_curl = nullptr;          // [ne][3][3]: surface curls of the local p1 basis
  int32_t *d_vstart = nullptr;       // [nv+1] CSR vertex -> (panel, local index)
  int32_t *d_vadj = nullptr;         // [3 ne][2]
  int storage_f32 = 0;
  hb::AsmParams params{};            // tables filled at creation
  hb::AsmParams launch{};            // per-call copy (outputs, ops), source of d_params
  hb::AsmParams *d_params = nullptr;
  hb::AsmParams *d_params_repr = nullptr;  // parameter copy read by the potential kernel
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  // solver workspace
  double *d_work = nullptr;
  size_t work_bytes = 0;
  double *d_v0inv = nullptr;         // inverse of V^0 (time marching; on a non-uniform grid
                                     // the inverses of all V^{k,k}, [nt][E_x][E_x])
  bool v0inv_valid = false;          // cleared whenever V is reassembled
  // learned preconditioner: row pattern, centroids, installed weights
  int32_t *d_pc_cols = nullptr;      // [ne][HB_PC_SLOTS]
  int8_t *d_pc_cls = nullptr;
  double *d_cent = nullptr;          // [ne][3]
  double *d_pc_M = nullptr;          // [ne][HB_PC_SLOTS]
  bool pc_active = false;
  float *d_pc_buf = nullptr;         // hb_precond_install: features, outputs, MLP workspace
  size_t pc_buf_n = 0;               // floats
  double *d_ir = nullptr;            // iterative refinement: x, r, correction
  size_t ir_bytes = 0;
  double *h_res = nullptr;           // pinned: GMRES residual estimates, read one step late
  int h_res_n = 0;
  hipEvent_t ev_step = nullptr, ev_prev = nullptr;
  double *d_reprq = nullptr;         // potentials: Q_{2k}(w) / (2k+1)! for p = 3/2
  double *d_apply = nullptr;         // per-group partial results of the Toeplitz apply
  size_t apply_bytes = 0;
  // non-uniform time grid (hb_create_nonuniform): nodes t_0 = 0 < ... < t_nt, packed blocks
  bool nu = false;
  std::vector<double> tnodes;
  int64_t nb = 0;                    // blocks per operator: nt (uniform) or nt (nt + 1) / 2
  hb::NuClosed *d_nu_closed = nullptr;
  int32_t n_nu_closed = 0, n_nu_taylor = 0;
  int32_t *d_nu_tout = nullptr, *d_nu_tdeg = nullptr;
  double rho2_sep = 0.0, rho2_touch = 0.0;  // squared distance bounds of separated and touching pairs
  double *d_nu_taylor = nullptr, *d_nu_tscale = nullptr;
  double *d_nu_h = nullptr;          // [nt]: step lengths h_k
  double *d_nu_t = nullptr;          // [nt + 1]: the time nodes t_k
};
