/*
 * heatbem.h -- C ABI of the MI355X (gfx950) space-time boundary element library for the 3D heat
 * equation, following Zapletal, Watschinger, Of, Merta, "Semi-analytic integration for a parallel
 * space-time boundary element method modeling the heat equation" (arXiv 2102.09811).
 *
 * Problem (Sec. 1): du/dt - alpha Laplace u = 0 in Omega x (0, T), u(x, 0) = 0, with Dirichlet
 * data on Sigma = dOmega x (0, T).  Omega's boundary is given as a closed triangle mesh Gamma_h
 * (E_x triangles, N_x vertices); (0, T) is cut into E_t uniform steps of length h = T / E_t
 * (tensor-product space-time mesh, Sec. 3).
 *
 * Conventions for every function:
 *   - Return value 0 (HB_OK) on success, a negative HB_E* code otherwise; hb_last_error() then
 *     holds a message.  No C++ exception crosses this boundary.
 *   - "Device pointer" arguments are addresses in the current HIP device's memory (for example
 *     the data_ptr() of a PyTorch tensor); "host pointer" arguments are ordinary process memory.
 *     The caller owns every pointer it passes; the library copies what it keeps.
 *   - Coefficient vectors are time-major (Sec. 3): entry [i * n + j] is time interval i
 *     (0-based) and spatial index j.  p0 x p0 vectors (Neumann datum w) have n = E_x;
 *     p1 x p0 vectors (Dirichlet datum g) have n = N_x.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.  Calls are
 *     stream-ordered: device outputs are complete when the stream reaches the end of the call.
 *     A context must not be used from two host threads at once.
 *   - Block storage: block d of an operator is a dense row-major matrix, blocks stored d-major:
 *     V: [E_t][E_x][E_x] (p0 test x p0 trial), K: [E_t][E_x][N_x] (p0 test x p1 trial).
 */
#ifndef HEATBEM_H
#define HEATBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define HB_OK 0
#define HB_EINVAL (-1)   /* bad argument (size, range, null pointer, unknown enum) */
#define HB_EMESH (-2)    /* mesh is not a valid closed 2-manifold triangulation */
#define HB_EORIENT (-3)  /* mesh orientation inconsistent or not outward */
#define HB_ENOMEM (-4)   /* device or host allocation failed */
#define HB_EHIP (-5)     /* a HIP runtime call failed */
#define HB_ENOCONV (-6)  /* iterative solver stopped before reaching the tolerance */
#define HB_ESTATE (-7)   /* call order violated (e.g. apply before assemble) */

/* ---- operators (bit flags for hb_assemble) ---- */
#define HB_OP_V 1u /* single-layer operator V_h, Sec. 3.1 */
#define HB_OP_K 2u /* double-layer operator K_h, Sec. 3.2 */
#define HB_OP_D 4u /* hypersingular operator D_h = D_h^1 + D_h^2, Sec. 3.3 (p1 x p1, N_x x N_x) */
#define HB_OP_KT 8u /* hb_apply only: K_h^T, the blocks of K_h transposed one by one (Sec. 3.2 remark
                      on K_T'), x: E_t x E_x, y: E_t x N_x */
#define HB_OP_V11 16u /* single layer between p1 functions, V_h^{11} (N_x x N_x), the matrix of the
                         paper's preconditioner for D_h (Sec. 6.1) */

/* ---- assembly precision ---- */
#define HB_PREC_FP64 0  /* every quadrature point in double precision */
#define HB_PREC_MIXED 1 /* separated pairs at large d in float (see hb_options.mixed_d_min) */

/* ---- element types for block copies / storage ---- */
#define HB_DTYPE_F64 0
#define HB_DTYPE_F32 1

typedef struct hb_ctx hb_ctx;

typedef struct hb_options {
  int32_t ss_order;     /* Gauss points per [0,1] coordinate of the regularised rules for
                           touching pairs (Sec. 5.2, eq. for the [0,1]^4 tensor rule); default 4,
                           range 1..8. */
  int32_t d_switch;     /* blocks d >= d_switch are integrated in time by the even Taylor
                           series of the hat-weighted heat kernel instead of second differences
                           of G^{dtau dt}; one of 3 (default), 8 or 16. */
  int32_t storage;      /* HB_DTYPE_F64 (default) or HB_DTYPE_F32 block storage. */
  int32_t mixed_d_min;  /* HB_PREC_MIXED: separated pairs at d >= d0 are evaluated in float,
                           where d0 is the first d >= max(mixed_d_min, d_switch) with d - d_switch
                           even (kernel value and a Taylor polynomial of degree 16 at d = 3 down
                           to 4 as d grows, truncation below 2e-9 of the block scale; double
                           accumulation); the closed-form blocks d < d_switch and all touching
                           pairs stay in double.  Default 3 (every Taylor block), minimum 2. */
  int32_t reserved[12]; /* must be zero */
} hb_options;

/* Fill *opt with the defaults above. */
void hb_default_options(hb_options *opt);

/* Host-only mesh check (no GPU use).  verts: host, [n_verts][3] float64; tris: host,
 * [n_tris][3] int32 vertex indices, counter-clockwise seen from outside.  Validates the mesh as
 * hb_create does and, if class_counts is not NULL, writes the number of ordered triangle pairs
 * sharing 0, 1, 2 and 3 vertices (separated, vertex, edge, identical; Sec. 3.1 "Galerkin
 * weights").  Returns HB_OK, HB_EINVAL, HB_EMESH or HB_EORIENT. */
int hb_check_mesh(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                  int64_t class_counts[4]);

/* Create a context for mesh Gamma_h, heat capacity alpha > 0, final time T > 0 and 1 <= n_t <= 65536
 * uniform steps (Sec. 3).  verts/tris are host pointers as for hb_check_mesh.  Validates the
 * mesh (closed, 2-manifold, consistently and outward oriented, no repeated or coincident
 * vertices, no degenerate triangle), classifies the triangle pairs, builds the quadrature tables
 * and uploads geometry to the current device.  opt may be NULL (defaults).  On success *out owns
 * its device memory until hb_destroy. */
int hb_create(hb_ctx **out, const double *verts, int64_t n_verts, const int32_t *tris,
              int64_t n_tris, double alpha, double T, int32_t n_t, const hb_options *opt);

/* Context on a non-uniform time grid (the paper's outlook, Sec. 7: the block integrals of
 * Sec. 3.1 and 3.2 at general interval endpoints).  t_nodes: host, n_t + 1 doubles,
 * 0 = t_0 < t_1 < ... < t_{n_t} = T (finite, strictly increasing), 1 <= n_t <= 4096; other
 * arguments as for hb_create (opt->storage must be HB_DTYPE_F64).  The Toeplitz structure is
 * lost: the operators are block lower triangular with n_t (n_t + 1) / 2 blocks
 *   V^{k,i}[l][m] = int_{I_k} int_{I_i} int_{gamma_l} int_{gamma_m} G_alpha(x - y, t - tau),
 * 0 <= i <= k < n_t (I_k = (t_k, t_{k+1})), and K^{k,i} likewise (p1 trial), block (k, i)
 * stored at index k (k + 1) / 2 + i.  Per point pair a block is either the four-term difference
 * G^{dtau dt}(t_k - t_i) + G^{dtau dt}(t_{k+1} - t_{i+1}) - G^{dtau dt}(t_{k+1} - t_i)
 * - G^{dtau dt}(t_k - t_{i+1}) (i < k; on the diagonal h_k G^{dtau}(r, 0) + G^{dtau dt}(r, 0)
 * - G^{dtau dt}(r, h_k)) or, where those terms would cancel, the even Taylor series of the
 * trapezoid-weighted kernel about the centre of its time support (same value, no cancellation).
 * On such a context: hb_assemble (HB_OP_V | HB_OP_K, HB_PREC_FP64), hb_get_blocks (d0, nd index
 * the packed blocks), hb_apply (HB_OP_V, HB_OP_K: y^k = sum_{i<=k} A^{k,i} x^i),
 * hb_rhs_dirichlet (M_h = blockdiag(h_k M_x)), hb_solve (HB_SOLVE_GMRES or HB_SOLVE_TIMEMARCH,
 * the latter with the inverses of every V^{k,k}, precond 0),
 * hb_eval_repr (closed-form time integrals over the intervals), hb_sizes, hb_last_assembly_ms,
 * hb_last_error and hb_destroy work; the other entry points return HB_EINVAL. */
int hb_create_nonuniform(hb_ctx **out, const double *verts, int64_t n_verts, const int32_t *tris,
                         int64_t n_tris, double alpha, const double *t_nodes, int32_t n_t,
                         const hb_options *opt);

/* 1 if ctx was created by hb_create_nonuniform, else 0 (also for NULL). */
int hb_is_nonuniform(const hb_ctx *ctx);

/* Release everything the context owns.  NULL is accepted.  Waits for the device. */
void hb_destroy(hb_ctx *ctx);

/* Message of the last failed call on ctx (or of the last failed hb_create / hb_check_mesh when
 * ctx is NULL).  Valid until the next call on the same context. */
const char *hb_last_error(const hb_ctx *ctx);

/* Sizes: writes E_x, N_x, E_t, and the number of touching ordered pairs. */
int hb_sizes(const hb_ctx *ctx, int64_t *n_tris, int64_t *n_verts, int32_t *n_t,
             int64_t *n_touching);

/* Assemble all E_t blocks of the operators in `ops` (HB_OP_V | HB_OP_K | HB_OP_D | HB_OP_V11) on
 * the device
 * (Sec. 3.1 eq. for V_h^d, Sec. 3.2 eq. for K_h^d; assembly order Sec. 5).  Each entry is the
 * spatial quadrature over a triangle pair of the exact temporal integral: Radon's 7-point rule
 * on each triangle for separated pairs, Sauter-Schwab [0,1]^4 rules of order opt.ss_order for
 * pairs sharing a vertex, an edge or the whole triangle.  precision: HB_PREC_FP64 or
 * HB_PREC_MIXED.  Block storage is allocated on first use and reused; the double layer also
 * keeps a workspace of the size of K (its separated-pair contributions of the transposed order,
 * folded into K at the end of the call).
 * HB_OP_D (Sec. 3.3): D_h^d = D_h^{1,d} + D_h^{2,d}, N_x x N_x blocks in the storage type.
 * D_h^{1,d} = T^T (alpha^2 V_h^d (x) I_3) T is formed from the assembled V_h and the surface
 * curls of the p1 basis (so V_h must be assembled before or in the same call, else HB_ESTATE);
 * D_h^{2,d} = int int n(x).n(y) phi_i phi_j D^{2,d} with the same rules as V_h, in double whatever
 * the precision argument.  D keeps a workspace of its own size.
 * HB_OP_V11: V_h^{11,d} = int int phi_i phi_j V^d (p1 x p1, N_x x N_x; the kernel, rules and
 * temporal forms of V_h), sharing D's workspace: assemblies of D and V11 on one context must not
 * overlap on different streams. */
int hb_assemble(hb_ctx *ctx, uint32_t ops, int32_t precision, void *stream);

/* Near field (the paper's outlook, Sec. 6.2: with a fast multipole method the formulae give the
 * near-field entries only).  hb_nearfield_pattern lists, per test panel l, the trial panels m whose
 * centroid lies within `radius` of l's, plus every panel touching l (shared vertex), sorted by m:
 * row_start[E_x + 1] (int64) and cols[nnz] (int32), host arrays, either may be NULL (nnz is always
 * written, so a first call with NULL arrays sizes them).  The pattern is kept for
 * hb_assemble_nearfield.  radius >= 0 and finite, else HB_EINVAL. */
int hb_nearfield_pattern(hb_ctx *ctx, double radius, int64_t *nnz, int64_t *row_start,
                         int32_t *cols);

/* Blocks of the near-field pairs of the last pattern, per pair: V[d][e] = V_h^d[l][cols[e]] and
 * K[d][e][k] = the contribution of panel cols[e] through its local vertex k (the p1 trial function
 * restricted to that panel; K_h^d[l][j] sums these over the panels at vertex j).  V: E_t x nnz,
 * K: E_t x nnz x 3, device float64.  Same kernels, rules and temporal forms as hb_assemble
 * (precision FP64).  HB_ESTATE without a pattern. */
int hb_assemble_nearfield(hb_ctx *ctx, double *V, double *K, void *stream);

/* Copy blocks d0 .. d0 + nd - 1 of op (HB_OP_V, HB_OP_K, HB_OP_D or HB_OP_V11) into dst (layout
 * [nd][rows][cols]
 * as the block storage), converting to dtype (HB_DTYPE_F64 / HB_DTYPE_F32).  dst is a device
 * pointer if dst_on_device != 0, else a host pointer (the copy is then synchronous). */
int hb_get_blocks(hb_ctx *ctx, uint32_t op, int32_t d0, int32_t nd, void *dst, int32_t dtype,
                  int32_t dst_on_device, void *stream);

/* Block lower-triangular Toeplitz product y^k = sum_{d=0}^{k} A^d x^{k-d} (Sec. 3.1 eq. for
 * V_h w; Sec. 3.2 eq. for K_h; Sec. 3.3) for op = HB_OP_V (x: E_t x E_x) or HB_OP_K (x: E_t x N_x),
 * y: E_t x E_x; op = HB_OP_D or HB_OP_V11 (x, y: E_t x N_x); op = HB_OP_KT (x: E_t x E_x, y: E_t x N_x; the
 * transposed blocks are formed once per assembly of K in a buffer of the size of K).
 * x, y: device pointers, float64, time-major, not overlapping.  Supports
 * E_t <= 256 (HB_EINVAL beyond); float block storage multiplies in float (x rounded to float) with
 * the partial sums added in double. */
int hb_apply(hb_ctx *ctx, uint32_t op, const double *x, double *y, void *stream);

/* hb_apply without allocation, for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product, kernels and arguments as hb_apply, with the partial results in a fixed 32 MiB device
 * array of the library (one per device, set up by hb_create) instead of a buffer the context
 * allocates.  The split over workgroups is narrowed until the partial results fit; HB_EINVAL when
 * one set of them, E_t x rows x element size (8 bytes, 4 with float storage), exceeds 32 MiB.
 * HB_OP_KT needs the transposed blocks formed by an hb_apply(HB_OP_KT) after the last assembly of
 * K (HB_ESTATE otherwise).  Every call on a device shares that device's array and leaves its
 * contents behind: calls that overlap on one device (two streams, or two host threads) race, so
 * the caller orders them. */
int hb_apply_noalloc(hb_ctx *ctx, uint32_t op, const double *x, double *y, void *stream);

/* Right-hand side of the Dirichlet system b = (1/2 M_h + K_h) g (Sec. 3.4) with
 * M_h = h blockdiag(M_x), M_x[l, j] = int phi^0_l phi^1_j.  g: device, E_t x N_x (coefficients
 * of Dirichlet data in the p1-space / p0-time space); b: device, E_t x E_x. */
int hb_rhs_dirichlet(hb_ctx *ctx, const double *g, double *b, void *stream);

/* Right-hand side of the Neumann system b = (1/2 M_h^T - K_h^T) psi (Sec. 3.4, the hypersingular
 * equation with the blockwise transposes).  psi: device, E_t x E_x (coefficients of the Neumann
 * datum alpha du/dn in the p0-space / p0-time space); b: device, E_t x N_x.  Needs K_h. */
int hb_rhs_neumann(hb_ctx *ctx, const double *psi, double *b, void *stream);

/* Solvers for V_h w = b (Sec. 3.4). */
#define HB_SOLVE_GMRES 0      /* unrestarted GMRES in double on the block system */
#define HB_SOLVE_TIMEMARCH 1  /* block forward substitution with the inverse of V_h^0 */
#define HB_SOLVE_MIXED_IR 2   /* iterative refinement: double residual b - V_h w, corrections from
                                 GMRES on a float copy of the blocks (float MFMA apply) */

typedef struct hb_solve_opts {
  int32_t method;   /* HB_SOLVE_* */
  int32_t max_iter; /* GMRES iteration cap over the whole solve (preconditioned phase, fallback
                       and restarts); per inner solve for HB_SOLVE_MIXED_IR, whose fallback then
                       gets max_iter more (default 500 if <= 0) */
  double tol;       /* relative residual ||b - V_h w|| / ||b|| target (default 1e-8 if <= 0) */
  int32_t precond;  /* GMRES methods: 1 = right-precondition with the sparse approximate inverse
                       installed by hb_precond_set, 0 = none */
  int32_t precond_max_iter; /* > 0: iteration cap of the preconditioned GMRES phase (for
                               HB_SOLVE_MIXED_IR: of all its inner iterations together) before
                               the plain double fallback takes over; 0 = no separate cap */
  int32_t reserved[6];
} hb_solve_opts;

typedef struct hb_solve_info {
  int32_t iterations;   /* GMRES iterations, summed over all phases (0 for time marching) */
  double rel_residual;  /* ||b - V_h w|| / ||b|| recomputed in double at the end of the solve */
  double seconds;       /* wall time of the solve (work queued before it on the stream is
                           drained before the clock starts) */
  int32_t refinements;  /* HB_SOLVE_MIXED_IR: outer refinement steps */
  int32_t fallback;     /* 1 if the preconditioned or mixed-precision phase ended above tol and
                           plain double GMRES continued from its iterate */
  int32_t restarts;     /* continuations after the first phase because the recomputed double
                           residual was above tol (GMRES restarts, repeated time marching) */
  int32_t reserved[5];
} hb_solve_info;

/* Solve V_h w = b for w.  b, w: device pointers, E_t x E_x, float64.  info may be NULL.
 * Residual contract (Sec. 6.1, relative accuracy in the double operator): HB_OK means that
 * ||b - V_h w|| / ||b|| <= tol, recomputed in double with the double blocks (float storage: the
 * float blocks with double accumulation) after the method has finished.  GMRES stops on its
 * Arnoldi estimate; if the recomputed residual is above tol, GMRES restarts from w on the
 * residual (within max_iter); a preconditioned (precond = 1) or HB_SOLVE_MIXED_IR phase that ends
 * above tol hands over to plain double GMRES from its iterate (info->fallback = 1); time marching
 * repeats its forward substitution on the residual at most three times.  Otherwise HB_ENOCONV,
 * with w holding the last iterate.  All methods use the block-Toeplitz product, so E_t <= 256.
 * The call returns once w and the residual check are complete on `stream` (it synchronizes with
 * the stream). */
int hb_solve(hb_ctx *ctx, const double *b, double *w, const hb_solve_opts *opts,
             hb_solve_info *info, void *stream);

/* Solve the Neumann system D_h u = b for u (Sec. 3.4) by unrestarted GMRES in double on the block
 * system (the paper uses FGMRES).  b, u: device pointers, E_t x N_x, float64.  opts: method must
 * be HB_SOLVE_GMRES (HB_EINVAL otherwise); tol and max_iter as for hb_solve; precond 1 applies
 * the operator preconditioner M_h^{-1} V_h^{11} M_h^{-1} from the right (Sec. 6.1: V_h^{11} as its
 * essential part; M_h = h blockdiag(M), M the p1 mass matrix, inverted once per context), which
 * needs HB_OP_V11 assembled.  Needs HB_OP_D assembled (HB_ESTATE).  info->rel_residual is
 * ||b - D_h u|| / ||b||; the residual contract, restarts and fallback (to GMRES without the
 * operator preconditioner) are those of hb_solve.  Returns once u is complete on `stream`. */
int hb_solve_neumann(hb_ctx *ctx, const double *b, double *u, const hb_solve_opts *opts,
                     hb_solve_info *info, void *stream);

/* Representation formula u = V~ w - W g (Sec. 2, potentials of Sec. 3.5) at P space-time points
 * pts[P][4] = (x, y, z, t), 0 <= t <= T, off Gamma_h (not checked; accuracy near Gamma_h is
 * the caller's concern).  w: E_t x E_x Neumann coefficients, g: E_t x N_x Dirichlet
 * coefficients, u: P outputs.  All device pointers, float64.  The spatial rule is the 7-point
 * rule of hb_assemble.  sl / dl may be NULL; otherwise they receive V~ w and W g.  Each point's
 * interval coefficients live in one workgroup's LDS, which bounds E_t at about 1650 (HB_EINVAL
 * beyond).  On a non-uniform context (hb_create_nonuniform) the rows of w and g belong to the
 * intervals [t_k, t_{k+1}] and every interval is integrated in closed form (the paper's outlook,
 * Sec. 7, with the time integrals of Sec. 3.5 over general intervals). */
int hb_eval_repr(hb_ctx *ctx, const double *pts, int64_t P, const double *w, const double *g,
                 double *u, double *sl, double *dl, void *stream);

/* ---- Learned preconditioner ----
 * M ~ (V_h^0)^{-1} restricted to the touching-panel pattern of every row (the panel itself, its
 * edge neighbours, then its vertex neighbours by centroid distance; at most HB_PC_SLOTS), used as
 * the block-diagonal right preconditioner diag(M, ..., M) of GMRES.  Its weights are predicted
 * per row by a 3-layer MLP from local data only (near-field V^0 entries and geometry) and
 * trained to minimise the row residual ||(M V^0)_l - e_l||^2 (a sparse approximate inverse).
 * This goes beyond the paper, whose solver is FGMRES without such a preconditioner (Sec. 6.1). */
#define HB_PC_SLOTS 16
#define HB_PC_SLOT_FEATURES 8
#define HB_PC_FEATURES (HB_PC_SLOTS * HB_PC_SLOT_FEATURES + 4)

typedef struct hb_mlp_dims {
  int32_t n_in, n_hidden, n_out; /* dense layers n_in -> n_hidden -> n_hidden -> n_out, tanh */
} hb_mlp_dims;

/* Row pattern: cols [E_x][HB_PC_SLOTS] int32 (panel indices, -1 = empty slot) and, if not NULL,
 * cls [E_x][HB_PC_SLOTS] int8 (3 itself, 2 edge, 1 vertex neighbour).  Device pointers. */
int hb_precond_pattern(hb_ctx *ctx, int32_t *cols, int8_t *cls, void *stream);

/* Row features [E_x][HB_PC_FEATURES] float (device).  Per slot: V^0[l,m]/V^0[l,l], class one-hot
 * (3), centroid distance / sqrt(area_l), area_m / area_l, n_l . n_m, present; then
 * sqrt(alpha h / area_l), its log, slot count / HB_PC_SLOTS, 1.  Needs V assembled. */
int hb_precond_features(hb_ctx *ctx, float *feats, void *stream);

/* Training data of the sparse approximate inverse, per row l, in the scaled unknowns
 * y = V^0[l,l] M[l, J]:  ||(M V^0)_l - e_l||^2 = y^T G y - 2 a^T y + 1 with
 * gram [E_x][S][S] = G and rhs [E_x][S] = a (device float, S = HB_PC_SLOTS); weights [E_x][S]
 * (may be NULL) receives the exact minimiser G^{-1} a.  Uses full rows of V^0. */
int hb_precond_spai(hb_ctx *ctx, float *gram, float *rhs, float *weights, void *stream);

/* Install the preconditioner from scaled weights [E_x][HB_PC_SLOTS] (device float):
 * M[l, cols[l][s]] = weights[l][s] / V^0[l,l].  weights = NULL uninstalls. */
int hb_precond_set(hb_ctx *ctx, const float *weights, void *stream);

/* MLP parameter count and forward / backward workspace size (floats) for a batch. Parameters
 * are one float array: W1 [H][I], b1 [H], W2 [H][H], b2 [H], W3 [O][H], b3 [O]. */
int64_t hb_mlp_num_params(const hb_mlp_dims *dims);
int64_t hb_mlp_work_floats(const hb_mlp_dims *dims, int64_t batch);

/* y [batch][O] = MLP(x [batch][I]); work keeps the activations for hb_mlp_backward.  Device. */
int hb_mlp_forward(const hb_mlp_dims *dims, const float *params, const float *x, int64_t batch,
                   float *y, float *work, void *stream);

/* grads (same layout as params) of sum over the batch of dy . y, given the work of the matching
 * hb_mlp_forward call.  Device pointers. */
int hb_mlp_backward(const hb_mlp_dims *dims, const float *params, const float *x, int64_t batch,
                    const float *work, const float *dy, float *grads, void *stream);

/* Loss of hb_precond_spai's quadratic form per row (rowloss, may be NULL) and the gradient of
 * its batch mean w.r.t. y (dy, may be NULL).  y, gram, rhs as above, rows entries.  Device. */
int hb_precond_loss(const float *y, const float *gram, const float *rhs, int64_t rows, float *dy,
                    float *rowloss, void *stream);

/* One Adam step p -= lr mhat / (sqrt(vhat) + eps) on n floats (step counts from 1).  Device. */
int hb_adam_step(float *params, const float *grads, float *m, float *v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int32_t step, void *stream);

/* ---- The learned preconditioner as one object: training, storage, installation ----
 * hb_pcnet holds a trained MLP (dims and parameters in device memory of the device current at
 * its creation).  Its input is a row's features (hb_precond_features, n_in = HB_PC_FEATURES) and
 * its output the row's scaled weights (n_out = HB_PC_SLOTS). */
typedef struct hb_pcnet hb_pcnet;

typedef struct hb_train_opts {
  int32_t epochs;       /* passes over all training rows (default 30 if <= 0) */
  int32_t batch;        /* rows per Adam step (default 2048 if <= 0; at most the row count); an
                           epoch's last partial batch is skipped */
  float lr;             /* Adam step size (default 1e-3 if <= 0; beta 0.9 / 0.999, eps 1e-8) */
  int32_t n_hidden;     /* width of both hidden layers (default 256 if <= 0, at most 4096) */
  uint64_t seed;        /* initial weights (Glorot uniform, zero biases) and every epoch's row
                           order (Fisher-Yates), both from the splitmix64 sequence of this seed */
  int32_t reserved[8];  /* must be zero */
} hb_train_opts;

/* Fill *opt with the defaults above (seed 0). */
void hb_default_train_opts(hb_train_opts *opt);

/* Train a network on the rows of n_ctx contexts (one mesh and alpha, h each; V assembled, else
 * HB_ESTATE): the sparse-approximate-inverse loss of hb_precond_spai, mean over each batch,
 * minimised by Adam with the library's forward / backward / loss / Adam kernels; shuffling,
 * batching (row gathers) and the epoch loop run in the library on `stream`.  Only V^0 is used, so
 * one-step contexts (T = h, n_t = 1) suffice.  epoch_loss (host, `epochs` floats, may be NULL)
 * receives each epoch's mean row loss.  On success *out is a new network owned by the caller
 * (hb_pcnet_destroy).  Device memory: 4 (HB_PC_FEATURES + HB_PC_SLOTS^2 + HB_PC_SLOTS) bytes per
 * training row plus the batch's activations; errors are reported on ctxs[0].  Synchronizes with
 * the stream once per epoch. */
int hb_precond_train(hb_ctx *const *ctxs, int32_t n_ctx, const hb_train_opts *opts,
                     hb_pcnet **out, float *epoch_loss, void *stream);

/* A network from given dims and parameters (host pointer, hb_mlp_num_params floats in the layout
 * of hb_mlp_forward).  HB_EINVAL unless n_in = HB_PC_FEATURES and n_out = HB_PC_SLOTS. */
int hb_pcnet_create(const hb_mlp_dims *dims, const float *params, hb_pcnet **out);

/* Dims and (if params, a host pointer, is not NULL) the parameters of net.  Synchronous. */
int hb_pcnet_get(const hb_pcnet *net, hb_mlp_dims *dims, float *params);

/* Write net to the file `path` (binary: the 8 bytes "HBPCNET1", int32 n_in, n_hidden, n_out,
 * int64 parameter count, then the float32 parameters, little-endian) / read such a file into a
 * new network on the current device.  HB_EINVAL for a missing, short or inconsistent file (message
 * in hb_last_error(NULL)). */
int hb_pcnet_save(const hb_pcnet *net, const char *path);
int hb_pcnet_load(const char *path, hb_pcnet **out);

/* Release a network (NULL accepted). */
void hb_pcnet_destroy(hb_pcnet *net);

/* Predict the preconditioner of ctx from its local data (features of its assembled V^0, then the
 * network's forward pass) and install it as hb_precond_set does.  Needs V (HB_ESTATE). */
int hb_precond_install(hb_ctx *ctx, const hb_pcnet *net, void *stream);

/* Durations in milliseconds of the kernels of the last hb_assemble on this context, measured
 * with HIP events on the caller's stream: [0] separated-pair kernel, [1] touching-pair kernels,
 * [2] whole call.  Calls hipEventSynchronize. */
int hb_last_assembly_ms(hb_ctx *ctx, double ms[3]);

/* Throughput of the vector ALU of the current device: microbenchmarks, not part of the method;
 * the ceilings the assembly and potential kernels are measured against.  out[0]: FP64 FMA rate
 * in TFLOP/s; out[1]: v_rsq_f64 rate in G/s (each step one v_rsq_f64 on the transcendental path,
 * which the square roots and reciprocals of the kernels use, and one v_add_f64); out[2]: FP32 FMA rate in TFLOP/s as this library is built
 * (without packed FP32 instructions).  Independent FMA or rsq chains in 4096 x 256 threads, the
 * best of five runs on `stream`, a few milliseconds each.  Allocates and frees 8 MiB of device
 * memory and synchronizes.  HB_EINVAL for out == NULL, HB_ENOMEM, HB_EHIP. */
int hb_measure_peaks(double out[3], void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HEATBEM_H */
