// Host runtime of the heat BEM library: mesh validation, triangle-pair classification,
// quadrature and Taylor tables, device uploads, and the C ABI entry points that manage a context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <unordered_map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "hb_internal.h"

namespace {

thread_local std::string g_err;  // last error of calls without a context

typedef long double ld;
const ld kPi = 3.141592653589793238462643383279502884L;

int fail(hb_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  else g_err = msg;
  return code;
}

}  // namespace

namespace hb {
void set_global_error(const std::string &msg) { g_err = msg; }
}  // namespace hb

namespace {

#define HB_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, e_ == hipErrorOutOfMemory ? HB_ENOMEM : HB_EHIP,                 \
                  std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

// ---------------------------------------------------------------------------------------------
// Mesh validation: closed, 2-manifold, consistently and outward oriented, no coincident vertices,
// no degenerate or repeated-vertex triangle, every vertex used.
// ---------------------------------------------------------------------------------------------
int validate_mesh(hb_ctx *c, const double *V, int64_t nv, const int32_t *T, int64_t ne) {
  if (!V || !T) return fail(c, HB_EINVAL, "null mesh pointer");
  if (nv < 4 || ne < 4) return fail(c, HB_EMESH, "a closed surface needs >= 4 vertices and triangles");
  if (ne > (int64_t)1 << 24 || nv > (int64_t)1 << 24)
    return fail(c, HB_EINVAL, "mesh too large");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(V[i])) return fail(c, HB_EMESH, "non-finite vertex coordinate");
  std::vector<int> used(nv, 0);
  double lo[3] = {V[0], V[1], V[2]}, hi[3] = {V[0], V[1], V[2]};
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], V[3 * i + k]); hi[k] = std::max(hi[k], V[3 * i + k]); }
  double diam2 = 0;
  for (int k = 0; k < 3; ++k) diam2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
  for (int64_t t = 0; t < ne; ++t) {
    int32_t a = T[3 * t], b = T[3 * t + 1], d = T[3 * t + 2];
    if (a < 0 || b < 0 || d < 0 || a >= nv || b >= nv || d >= nv)
      return fail(c, HB_EMESH, "triangle " + std::to_string(t) + " has an out-of-range vertex index");
    if (a == b || b == d || a == d)
      return fail(c, HB_EMESH, "triangle " + std::to_string(t) + " repeats a vertex");
    used[a] = used[b] = used[d] = 1;
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) { e1[k] = V[3 * b + k] - V[3 * a + k]; e2[k] = V[3 * d + k] - V[3 * a + k]; }
    double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
           cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (cx * cx + cy * cy + cz * cz <= 1e-24 * diam2 * diam2)
      return fail(c, HB_EMESH, "triangle " + std::to_string(t) + " is degenerate");
  }
  for (int64_t i = 0; i < nv; ++i)
    if (!used[i]) return fail(c, HB_EMESH, "vertex " + std::to_string(i) + " belongs to no triangle");
  // coincident vertices with different indices
  std::vector<int64_t> ord(nv);
  for (int64_t i = 0; i < nv; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
    for (int k = 0; k < 3; ++k)
      if (V[3 * x + k] != V[3 * y + k]) return V[3 * x + k] < V[3 * y + k];
    return x < y;
  });
  for (int64_t i = 1; i < nv; ++i)
    if (V[3 * ord[i]] == V[3 * ord[i - 1]] && V[3 * ord[i] + 1] == V[3 * ord[i - 1] + 1] &&
        V[3 * ord[i] + 2] == V[3 * ord[i - 1] + 2])
      return fail(c, HB_EMESH, "vertices " + std::to_string(ord[i - 1]) + " and " +
                                   std::to_string(ord[i]) + " coincide");
  // every undirected edge exactly twice, once in each direction
  std::map<std::pair<int32_t, int32_t>, std::pair<int, int>> edges;  // (min,max) -> (+dir, -dir)
  for (int64_t t = 0; t < ne; ++t)
    for (int k = 0; k < 3; ++k) {
      int32_t p = T[3 * t + k], q = T[3 * t + (k + 1) % 3];
      auto &e = edges[{std::min(p, q), std::max(p, q)}];
      if (p < q) e.first++;
      else e.second++;
    }
  for (auto &kv : edges) {
    int tot = kv.second.first + kv.second.second;
    if (tot != 2)
      return fail(c, HB_EMESH, "edge (" + std::to_string(kv.first.first) + "," +
                                   std::to_string(kv.first.second) + ") belongs to " +
                                   std::to_string(tot) + " triangles (mesh not closed/manifold)");
    if (kv.second.first != 1)
      return fail(c, HB_EORIENT, "inconsistent orientation at edge (" +
                                     std::to_string(kv.first.first) + "," +
                                     std::to_string(kv.first.second) + ")");
  }
  // outward: positive enclosed volume
  ld vol = 0;
  for (int64_t t = 0; t < ne; ++t) {
    const double *a = V + 3 * T[3 * t], *b = V + 3 * T[3 * t + 1], *d = V + 3 * T[3 * t + 2];
    vol += (ld)a[0] * ((ld)b[1] * d[2] - (ld)b[2] * d[1]) - (ld)a[1] * ((ld)b[0] * d[2] - (ld)b[2] * d[0]) +
           (ld)a[2] * ((ld)b[0] * d[1] - (ld)b[1] * d[0]);
  }
  if (!(vol > 0)) return fail(c, HB_EORIENT, "triangles are oriented inward (negative volume)");
  return HB_OK;
}

// ---------------------------------------------------------------------------------------------
// Pair classification by shared vertex indices.  For a touching ordered pair (test l, trial m) the
// rule expects the shared vertices first and in the same order in both panels:
//   identical: both panels in the test's order;  edge: (s, t, rest) in both;
//   vertex: (s, then the other two in the panel's cyclic order) in both.
// ---------------------------------------------------------------------------------------------
struct Adjacency {
  std::vector<int64_t> start;
  std::vector<int32_t> tri;
};

Adjacency vertex_triangles(const int32_t *T, int64_t nv, int64_t ne) {
  Adjacency A;
  A.start.assign(nv + 1, 0);
  for (int64_t i = 0; i < 3 * ne; ++i) A.start[T[i] + 1]++;
  for (int64_t i = 0; i < nv; ++i) A.start[i + 1] += A.start[i];
  A.tri.resize(3 * ne);
  std::vector<int64_t> fill(A.start.begin(), A.start.end() - 1);
  for (int64_t t = 0; t < ne; ++t)
    for (int k = 0; k < 3; ++k) A.tri[fill[T[3 * t + k]]++] = (int32_t)t;
  return A;
}

// Local orders (pl, pm) of the vertices of panels l and m; returns the number of shared vertices.
int pair_order(const int32_t *tl, const int32_t *tm, int pl[3], int pm[3]) {
  int where[3] = {-1, -1, -1};  // where[i]: local index in m of vertex i of l
  int ns = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (tl[i] == tm[j]) { where[i] = j; ++ns; }
  if (ns == 3) {
    for (int i = 0; i < 3; ++i) { pl[i] = i; pm[i] = where[i]; }
  } else if (ns == 2) {
    int k = 0;
    for (int i = 0; i < 3; ++i)
      if (where[i] >= 0) { pl[k] = i; pm[k] = where[i]; ++k; }
    for (int i = 0; i < 3; ++i)
      if (where[i] < 0) pl[2] = i;
    pm[2] = 3 - pm[0] - pm[1];
  } else if (ns == 1) {
    int i0 = 0;
    while (where[i0] < 0) ++i0;
    pl[0] = i0; pl[1] = (i0 + 1) % 3; pl[2] = (i0 + 2) % 3;
    int j0 = where[i0];
    pm[0] = j0; pm[1] = (j0 + 1) % 3; pm[2] = (j0 + 2) % 3;
  }
  return ns;
}

void count_classes(const int32_t *T, int64_t nv, int64_t ne, int64_t counts[4],
                   std::vector<hb::TouchPair> *out, const double *V) {
  Adjacency A = vertex_triangles(T, nv, ne);
  for (int k = 0; k < 4; ++k) counts[k] = 0;
  std::vector<int64_t> seen(ne, -1);
  for (int64_t l = 0; l < ne; ++l) {
    const int32_t *tl = T + 3 * l;
    for (int k = 0; k < 3; ++k)
      for (int64_t s = A.start[tl[k]]; s < A.start[tl[k] + 1]; ++s) {
        int32_t m = A.tri[s];
        if (seen[m] == l) continue;
        seen[m] = l;
        int pl[3], pm[3];
        const int32_t *tm = T + 3 * m;
        int ns = pair_order(tl, tm, pl, pm);
        counts[ns]++;
        if (out) {
          hb::TouchPair p{};
          p.l = (int32_t)l; p.m = m; p.cls = ns;
          for (int j = 0; j < 3; ++j) p.vtx[j] = tm[pm[j]];
          for (int j = 0; j < 3; ++j) p.vtxl[j] = tl[pl[j]];
          for (int cc = 0; cc < 3; ++cc) {
            p.E1[cc] = V[3 * tl[pl[1]] + cc] - V[3 * tl[pl[0]] + cc];
            p.E2[cc] = V[3 * tl[pl[2]] + cc] - V[3 * tl[pl[1]] + cc];
            p.F1[cc] = V[3 * tm[pm[1]] + cc] - V[3 * tm[pm[0]] + cc];
            p.F2[cc] = V[3 * tm[pm[2]] + cc] - V[3 * tm[pm[1]] + cc];
          }
          out->push_back(p);
        }
      }
  }
  counts[0] = ne * ne - counts[1] - counts[2] - counts[3];
}

// ---------------------------------------------------------------------------------------------
// Quadrature and series tables (long double on the host, rounded once).
// ---------------------------------------------------------------------------------------------
// Gauss-Legendre on [0,1]: roots of P_n by Newton from Tricomi's initial guesses.
void legendre01(int n, std::vector<ld> &x, std::vector<ld> &w) {
  x.resize(n);
  w.resize(n);
  for (int k = 1; k <= n; ++k) {
    ld th = kPi * (4.0L * k - 1.0L) / (4.0L * n + 2.0L);
    ld t = (1.0L - (n - 1.0L) / (8.0L * n * n * n)) * cosl(th);
    ld pn = 0, dpn = 0;
    for (int it = 0; it < 60; ++it) {
      ld pm1 = 1.0L, p = t;  // P_0, P_1
      for (int j = 2; j <= n; ++j) {
        ld pj = ((2 * j - 1) * t * p - (j - 1) * pm1) / j;
        pm1 = p;
        p = pj;
      }
      if (n == 1) { p = t; pm1 = 1.0L; }
      pn = p;
      dpn = n * (pm1 - t * p) / (1.0L - t * t);
      ld step = pn / dpn;
      t -= step;
      if (fabsl(step) <= 1e-20L * fabsl(t) + 1e-22L) break;
    }
    {
      ld pm1 = 1.0L, p = t;
      for (int j = 2; j <= n; ++j) {
        ld pj = ((2 * j - 1) * t * p - (j - 1) * pm1) / j;
        pm1 = p;
        p = pj;
      }
      if (n == 1) { p = t; pm1 = 1.0L; }
      dpn = n * (pm1 - t * p) / (1.0L - t * t);
    }
    x[k - 1] = (1.0L + t) / 2.0L;
    w[k - 1] = 1.0L / ((1.0L - t * t) * dpn * dpn);
  }
}

// Regularised rules (Sauter & Schwab, Sec. 5.2 of their book) written as the coefficients of
// r = x - y in the edge vectors, so the kernel never subtracts two nearby points:
//   r = c1 E1 + c2 E2 + c3 F1 + c4 F2,  E1 = a1-a0, E2 = a2-a1 (test), F1 = b1-b0, F2 = b2-b1.
// Reference panel {0 <= s2 <= s1 <= 1}, chi(s) = v0 + s1 (v1-v0) + s2 (v2-v1).  Each entry holds
// (c1, c2, c3, c4, weight * Jacobian, trial barycentrics (1-y1, y1-y2, y2), test barycentrics
// (1-x1, x1-x2, x2)).
struct SSNode { ld c[4], w, lam[3], lamx[3]; };

void ss_nodes(int cls, int M, std::vector<SSNode> &out) {
  std::vector<ld> g, gw;
  legendre01(M, g, gw);
  out.clear();
  int nmaps = cls == 3 ? 6 : (cls == 2 ? 5 : 2);
  for (int s = 0; s < nmaps; ++s)
    for (int i0 = 0; i0 < M; ++i0)
      for (int i1 = 0; i1 < M; ++i1)
        for (int i2 = 0; i2 < M; ++i2)
          for (int i3 = 0; i3 < M; ++i3) {
            ld xi = g[i0], a = g[i1], b = g[i2], e = g[i3];
            ld wt = gw[i0] * gw[i1] * gw[i2] * gw[i3];
            ld x1, x2, y1, y2, d1, d2, J;  // d1 = x1 - y1, d2 = x2 - y2 in product form
            if (cls == 3) {
              J = xi * xi * xi * a * a * b;
              switch (s) {
                case 0: x1 = xi; x2 = xi * (1 - a + a * b); y1 = xi * (1 - a * b * e); y2 = xi * (1 - a);
                        d1 = xi * a * b * e; d2 = xi * a * b; break;
                case 1: x1 = xi * (1 - a * b * e); x2 = xi * (1 - a); y1 = xi; y2 = xi * (1 - a + a * b);
                        d1 = -xi * a * b * e; d2 = -xi * a * b; break;
                case 2: x1 = xi; x2 = xi * a * (1 - b + b * e); y1 = xi * (1 - a * b); y2 = xi * a * (1 - b);
                        d1 = xi * a * b; d2 = xi * a * b * e; break;
                case 3: x1 = xi * (1 - a * b); x2 = xi * a * (1 - b); y1 = xi; y2 = xi * a * (1 - b + b * e);
                        d1 = -xi * a * b; d2 = -xi * a * b * e; break;
                case 4: x1 = xi * (1 - a * b * e); x2 = xi * a * (1 - b * e); y1 = xi; y2 = xi * a * (1 - b);
                        d1 = -xi * a * b * e; d2 = xi * a * b * (1 - e); break;
                default: x1 = xi; x2 = xi * a * (1 - b); y1 = xi * (1 - a * b * e); y2 = xi * a * (1 - b * e);
                         d1 = xi * a * b * e; d2 = -xi * a * b * (1 - e); break;
              }
              out.push_back({{d1, d2, 0, 0}, wt * J, {1 - y1, y1 - y2, y2}, {1 - x1, x1 - x2, x2}});
            } else if (cls == 2) {
              J = xi * xi * xi * a * a * (s == 0 ? 1.0L : b);
              switch (s) {
                case 0: x1 = xi; x2 = xi * a * e; y1 = xi * (1 - a * b); y2 = xi * a * (1 - b);
                        d1 = xi * a * b; break;
                case 1: x1 = xi; x2 = xi * a; y1 = xi * (1 - a * b * e); y2 = xi * a * b * (1 - e);
                        d1 = xi * a * b * e; break;
                case 2: x1 = xi * (1 - a * b); x2 = xi * a * (1 - b); y1 = xi; y2 = xi * a * b * e;
                        d1 = -xi * a * b; break;
                case 3: x1 = xi * (1 - a * b * e); x2 = xi * a * b * (1 - e); y1 = xi; y2 = xi * a;
                        d1 = -xi * a * b * e; break;
                default: x1 = xi * (1 - a * b * e); x2 = xi * a * (1 - b * e); y1 = xi; y2 = xi * a * b;
                         d1 = -xi * a * b * e; break;
              }
              // shared edge: F1 == E1, so r = (x1 - y1) E1 + x2 E2 - y2 F2
              out.push_back({{d1, x2, 0, -y2}, wt * J, {1 - y1, y1 - y2, y2}, {1 - x1, x1 - x2, x2}});
            } else {
              J = xi * xi * xi * b;
              if (s == 0) { x1 = xi; x2 = xi * a; y1 = xi * b; y2 = xi * b * e; }
              else { x1 = xi * b; x2 = xi * b * e; y1 = xi; y2 = xi * a; }
              out.push_back({{x1, x2, -y1, -y2}, wt * J, {1 - y1, y1 - y2, y2}, {1 - x1, x1 - x2, x2}});
            }
          }
}

// Even Taylor series of the hat-weighted kernel in time.  With s = d h and w = rho^2/(4 alpha s),
//   int_{-h}^{h} (h - |u|) f(s + u) du = sum_k 2 h^{2k+2}/(2k+2)! f^{(2k)}(s),
// and for f(s) = s^{-p} exp(-a/s):  f^{(n)}(s) = s^{-p-n} exp(-w) Q_n(w),
//   Q_0 = 1,  Q_{n+1}(w) = (w - n - p) Q_n(w) - w Q_n'(w).
// So the block integral is h^2 f(s) P_d(w) with P_d(w) = sum_k 2/(2k+2)! d^{-2k} Q_{2k}(w),
// truncated at k = kTaylorDeg/2 (p = 3/2 for G, p = 5/2 for alpha dG/dn).
void taylor_poly(ld p, int d, ld out[hb::kTaylorN], int deg = hb::kTaylorDeg) {
  const int K = deg / 2;
  std::vector<std::vector<ld>> Q(2 * K + 1);
  Q[0] = {1.0L};
  for (int n = 0; n < 2 * K; ++n) {
    const auto &q = Q[n];
    std::vector<ld> r(q.size() + 1, 0.0L);
    for (size_t j = 0; j < q.size(); ++j) {
      r[j + 1] += q[j];
      r[j] -= (n + p) * q[j];
      r[j] -= (ld)j * q[j];
    }
    Q[n + 1] = r;
  }
  for (int j = 0; j < hb::kTaylorN; ++j) out[j] = 0;
  ld fact = 2.0L, dpow = 1.0L;  // (2k+2)! starting at k = 0, d^{-2k}
  for (int k = 0; k <= K; ++k) {
    if (k > 0) fact *= (ld)(2 * k + 1) * (ld)(2 * k + 2);
    ld coef = 2.0L / fact * dpow;
    for (size_t j = 0; j < Q[2 * k].size(); ++j) out[j] += coef * Q[2 * k][j];
    dpow /= (ld)d * (ld)d;
  }
}

// Odd Taylor series of D^{2,d} (Sec. 3.3): alpha h int_{-1}^{1} sgn(u) G(r, (d+u) h) du
//   = alpha h G(r, dh) sum_k 2 d^{-(2k+1)} Q_{2k+1}(w) / (2k+2)!  (Q_n as above, p = 3/2),
// truncated at k = deg/2: a polynomial of degree deg + 1 in w.
void taylor_poly_odd(int d, int deg, ld *out, int len) {
  const int K = deg / 2;
  const ld p = 1.5L;
  std::vector<std::vector<ld>> Q(2 * K + 2);
  Q[0] = {1.0L};
  for (int n = 0; n < 2 * K + 1; ++n) {
    const auto &q = Q[n];
    std::vector<ld> r(q.size() + 1, 0.0L);
    for (size_t j = 0; j < q.size(); ++j) {
      r[j + 1] += q[j];
      r[j] -= (n + p) * q[j];
      r[j] -= (ld)j * q[j];
    }
    Q[n + 1] = r;
  }
  for (int j = 0; j < len; ++j) out[j] = 0;
  ld fact = 2.0L, dpow = 1.0L / (ld)d;  // (2k+2)!, d^{-(2k+1)}
  for (int k = 0; k <= K; ++k) {
    if (k > 0) fact *= (ld)(2 * k + 1) * (ld)(2 * k + 2);
    const ld coef = 2.0L / fact * dpow;
    for (size_t j = 0; j < Q[2 * k + 1].size() && (int)j < len; ++j) out[j] += coef * Q[2 * k + 1][j];
    dpow /= (ld)d * (ld)d;
  }
}

// Shortest length N of the series polynomial c[0 .. len-1] in w whose dropped terms stay below
// tol |c_0| for every w in [0, wmax], for the polynomial and for its derivative (the double-layer
// kernel takes P - P'), both weighted by the factor e^{-w} the kernels multiply with.  Bounded
// cell by cell on a grid: on [w_i, w_{i+1}] the powers are at most their values at w_{i+1} and
// e^{-w} at most e^{-w_i}.  Per cell the tail is accumulated from the top term down; the first
// term at which it passes the bound is the last one the cell needs.
int taylor_len(const ld *c, int len, ld wmax, ld tol) {
  constexpr int kCells = 256;
  const ld bound = tol * fabsl(c[0]);
  int need = 1;
  for (int i = 0; i < kCells && need < len; ++i) {
    const ld w0 = wmax * i / kCells, w1 = wmax * (i + 1) / kCells;
    const ld lim = bound / expl(-w0);  // +inf once e^{-w0} is 0: nothing is needed there
    ld pw[hb::kTaylorN + 1];
    pw[0] = 1.0L;
    for (int n = 1; n < len; ++n) pw[n] = pw[n - 1] * w1;
    ld tail = 0.0L;
    for (int n = len - 1; n >= 1; --n) {
      tail += fabsl(c[n]) * (pw[n] + (ld)n * pw[n - 1]);
      if (!(tail <= lim)) {
        need = std::max(need, n + 1);
        break;
      }
    }
  }
  return need;
}

int upload(hb_ctx *c, void **dst, const void *src, size_t bytes) {
  HB_HIP(c, hipMalloc(dst, bytes));
  HB_HIP(c, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return HB_OK;
}

int build_tables(hb_ctx *c) {
  using namespace hb;
  AsmParams &p = c->params;
  p.ne = (int32_t)c->ne;
  p.nv = (int32_t)c->nv;
  p.nt = c->nt;
  p.dsw = c->opt.d_switch;
  p.alpha = c->alpha;
  p.h = c->h;
  ld al = c->alpha, h = c->h;
  for (int i = 0; i <= kMaxClosed; ++i) {
    ld delta = i * h;
    ld sq = sqrtl(al * delta);
    p.lv.c[i] = i == 0 ? 0.0 : (double)(1.0L / (2.0L * sq));
    p.lv.s2[i] = (double)(2.0L * al * delta);
    p.lv.s1[i] = (double)(2.0L * sq / sqrtl(kPi));
    p.lv.t2[i] = (double)(4.0L * sq / sqrtl(kPi));
  }
  // small-z series: sqrt(pi) A(z) = 2/z + z sum a_n z^{2n},  a_n = (-1)^n 2/((n+1)!(2n+1)(2n+3))
  //                 sqrt(pi) B(z) = 4 z sum b_n z^{2n},     b_n = (-1)^n /(n!(2n+1)(2n+3))
  ld fact = 1.0L;  // n!
  for (int n = 0; n < kSeriesN; ++n) {
    if (n > 0) fact *= n;
    ld sgn = (n % 2) ? -1.0L : 1.0L;
    p.serA[n] = (double)(sgn * 2.0L / (fact * (n + 1) * (2 * n + 1) * (2 * n + 3)));
    p.serB[n] = (double)(sgn / (fact * (2 * n + 1) * (2 * n + 3)));
  }
  // Radon's degree-5 rule: centroid, and the orbits of (a, a, 1-2a) for a = (6 -+ sqrt 15)/21
  ld r15 = sqrtl(15.0L);
  ld a1 = (6.0L - r15) / 21.0L, a2 = (6.0L + r15) / 21.0L;
  ld bary[7][3] = {{1 / 3.0L, 1 / 3.0L, 1 / 3.0L},
                   {1 - 2 * a1, a1, a1}, {a1, 1 - 2 * a1, a1}, {a1, a1, 1 - 2 * a1},
                   {1 - 2 * a2, a2, a2}, {a2, 1 - 2 * a2, a2}, {a2, a2, 1 - 2 * a2}};
  ld wts[7] = {0.225L, (155.0L - r15) / 1200.0L, (155.0L - r15) / 1200.0L,
               (155.0L - r15) / 1200.0L, (155.0L + r15) / 1200.0L,
               (155.0L + r15) / 1200.0L, (155.0L + r15) / 1200.0L};
  for (int q = 0; q < 7; ++q) {
    p.w7[q] = (double)wts[q];
    for (int k = 0; k < 3; ++k) p.lam7[q][k] = (double)bary[q][k];
  }
  p.kV = (double)(1.0L / (8.0L * kPi * al * al));
  p.kVs = (double)(h / (4.0L * kPi * al));
  p.kK = (double)(1.0L / (8.0L * kPi * al));
  p.kKs = (double)(h / (4.0L * kPi));

  // Taylor tables for d >= dsw.  The series converges like d^{-2k}: the truncation order is
  // chosen per d so that the dropped terms stay below ~2e-16 of the block scale (double path) or
  // ~1e-9 (float path), which shortens the polynomial as d grows.  The separated-pair kernel
  // evaluates blocks in pairs (dsw, dsw+1), (dsw+2, dsw+3), ... with one polynomial length, so
  // each block takes the degree of the first block of its pair.
  auto deg64 = [](int d) {
    return d < 4 ? 28 : d < 5 ? 24 : d < 6 ? 20 : d < 7 ? 18 : d < 8 ? 16 : d < 12 ? 14
         : d < 16 ? 12 : d < 32 ? 10 : d < 64 ? 8 : 6;
  };
  auto deg32 = [](int d) {
    return d < 4 ? 16 : d < 5 ? 12 : d < 7 ? 10 : d < 12 ? 8 : d < 24 ? 6 : 4;
  };
  auto pass_start = [&](int d) { return d - ((d - p.dsw) & 1); };
  std::vector<double> tay((size_t)c->nt * 2 * kTaylorN, 0.0), tsc((size_t)c->nt * 3, 0.0);
  std::vector<float> tay32((size_t)c->nt * 2 * kTaylorN32, 0.0f);
  std::vector<int32_t> tdeg((size_t)c->nt * 2, 0), tlen_sep((size_t)c->nt, 0),
      tlen_touch((size_t)c->nt, 0);
  // At block d a pair at distance rho evaluates the polynomial at w = rho^2 c_d, c_d =
  // 1 / (4 alpha d h).  Bounding rho bounds w, and where w stays small the terms of high power in
  // w are negligible: each pass then uses the shortest prefix of the same polynomial whose
  // dropped part stays below 1e-16 of the block scale (on top of the truncation of the series
  // itself).  Separated pairs: rho is at most twice the largest distance of a vertex from the
  // centre of the mesh's bounding box.  Touching pairs: rho is at most the largest vertex distance
  // of two triangles that share a vertex.
  ld rho2_sep = 0.0L;
  {
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = c->verts[k];
    for (size_t v = 0; v < c->verts.size() / 3; ++v)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], c->verts[3 * v + k]);
        hi[k] = std::max(hi[k], c->verts[3 * v + k]);
      }
    for (size_t v = 0; v < c->verts.size() / 3; ++v) {
      ld r2 = 0.0L;
      for (int k = 0; k < 3; ++k) {
        const ld x = (ld)c->verts[3 * v + k] - 0.5L * ((ld)lo[k] + hi[k]);
        r2 += x * x;
      }
      rho2_sep = std::max(rho2_sep, 4.0L * r2);
    }
  }
  ld rho2_touch = 0.0L;
  for (const TouchPair &tp : c->touch)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double *x = &c->verts[3 * c->tris[3 * tp.l + i]], *y = &c->verts[3 * c->tris[3 * tp.m + j]];
        ld r2 = 0.0L;
        for (int k = 0; k < 3; ++k) r2 += ((ld)x[k] - y[k]) * ((ld)x[k] - y[k]);
        rho2_touch = std::max(rho2_touch, r2);
      }
  c->rho2_sep = (double)rho2_sep;
  c->rho2_touch = (double)rho2_touch;
  for (int d = std::max(1, p.dsw); d < c->nt; ++d) {
    ld pv[kTaylorN], pk[kTaylorN];
    tdeg[2 * d] = deg64(pass_start(d));
    tdeg[2 * d + 1] = deg32(pass_start(d));
    taylor_poly(1.5L, d, pv, tdeg[2 * d]);
    taylor_poly(2.5L, d, pk, tdeg[2 * d]);
    {
      const ld cd = 1.0L / (4.0L * al * d * h);
      int32_t &Ls = tlen_sep[pass_start(d)], &Lt = tlen_touch[pass_start(d)];
      Ls = std::max<int32_t>(Ls, taylor_len(pv, tdeg[2 * d] + 1, rho2_sep * cd, 1e-16L));
      Lt = std::max<int32_t>(Lt, taylor_len(pv, tdeg[2 * d] + 1, rho2_touch * cd, 1e-16L));
    }
    for (int j = 0; j < kTaylorN; ++j) {
      tay[((size_t)d * 2 + 0) * kTaylorN + j] = (double)pv[j];
      tay[((size_t)d * 2 + 1) * kTaylorN + j] = (double)pk[j];
    }
    taylor_poly(1.5L, d, pv, tdeg[2 * d + 1]);
    taylor_poly(2.5L, d, pk, tdeg[2 * d + 1]);
    for (int j = 0; j < kTaylorN32; ++j) {
      tay32[((size_t)d * 2 + 0) * kTaylorN32 + j] = (float)pv[j];
      tay32[((size_t)d * 2 + 1) * kTaylorN32 + j] = (float)pk[j];
    }
    ld s = d * h;
    tsc[3 * d + 0] = (double)(h * h * powl(4.0L * kPi * al * s, -1.5L));
    tsc[3 * d + 1] = (double)(h * h / (16.0L * powl(kPi * al, 1.5L) * powl(s, 2.5L)));
    tsc[3 * d + 2] = (double)(1.0L / (4.0L * al * s));
  }
  int rc;
  if ((rc = upload(c, (void **)&c->d_taylor, tay.data(), tay.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, (void **)&c->d_tscale, tsc.data(), tsc.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, (void **)&c->d_taylor32, tay32.data(), tay32.size() * sizeof(float)))) return rc;
  if ((rc = upload(c, (void **)&c->d_tdeg, tdeg.data(), tdeg.size() * sizeof(int32_t)))) return rc;
  for (auto *tl : {&tlen_sep, &tlen_touch})
    for (int32_t &L : *tl) {
      if (L == 0) continue;
      for (int n : kPolyLens)
        if (n >= L) { L = n; break; }
      L = std::min<int32_t>(L, kTaylorN);
    }
  if ((rc = upload(c, (void **)&c->d_tlen_sep, tlen_sep.data(), tlen_sep.size() * sizeof(int32_t))))
    return rc;
  if ((rc = upload(c, (void **)&c->d_tlen_touch, tlen_touch.data(), tlen_touch.size() * sizeof(int32_t))))
    return rc;


  // geometry SoA: far-rule nodes, normal, area
  size_t ne = (size_t)c->ne;
  std::vector<double> geom(25 * ne);
  c->area.resize(ne);
  c->normal.resize(3 * ne);
  for (size_t t = 0; t < ne; ++t) {
    const double *v[3] = {&c->verts[3 * c->tris[3 * t]], &c->verts[3 * c->tris[3 * t + 1]],
                          &c->verts[3 * c->tris[3 * t + 2]]};
    ld e1[3], e2[3];
    for (int k = 0; k < 3; ++k) { e1[k] = (ld)v[1][k] - v[0][k]; e2[k] = (ld)v[2][k] - v[0][k]; }
    ld cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                e1[0] * e2[1] - e1[1] * e2[0]};
    ld nn = sqrtl(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    c->area[t] = (double)(0.5L * nn);
    for (int k = 0; k < 3; ++k) c->normal[3 * t + k] = (double)(cr[k] / nn);
    for (int q = 0; q < 7; ++q)
      for (int k = 0; k < 3; ++k)
        geom[(q * 3 + k) * ne + t] =
            (double)(bary[q][0] * v[0][k] + bary[q][1] * v[1][k] + bary[q][2] * v[2][k]);
    for (int k = 0; k < 3; ++k) geom[(21 + k) * ne + t] = c->normal[3 * t + k];
    geom[24 * ne + t] = c->area[t];
  }
  if ((rc = upload(c, (void **)&c->d_geom, geom.data(), geom.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, (void **)&c->d_tris, c->tris.data(), c->tris.size() * sizeof(int32_t)))) return rc;
  std::vector<double> mass(3 * ne);
  for (size_t t = 0; t < ne; ++t)
    for (int k = 0; k < 3; ++k) mass[3 * t + k] = c->area[t] / 3.0;
  if ((rc = upload(c, (void **)&c->d_mass, mass.data(), mass.size() * sizeof(double)))) return rc;

  // touching pairs (class 3, 2, 1 contiguous), with normals and area factors
  std::stable_sort(c->touch.begin(), c->touch.end(),
                   [](const TouchPair &x, const TouchPair &y) { return x.cls > y.cls; });
  for (auto &tp : c->touch) {
    for (int k = 0; k < 3; ++k) tp.n[k] = c->normal[3 * tp.m + k];
    tp.scale = 4.0 * c->area[tp.l] * c->area[tp.m];
    tp.nn = 0.0;
    for (int k = 0; k < 3; ++k) tp.nn += c->normal[3 * tp.l + k] * c->normal[3 * tp.m + k];
  }
  if (!c->touch.empty())
    if ((rc = upload(c, (void **)&c->d_touch, c->touch.data(), c->touch.size() * sizeof(TouchPair))))
      return rc;
  // the touching-pair assembly takes every identical and edge pair, and each pair sharing one
  // vertex once (l < m, marked ~index) for both of its orders
  {
    std::vector<int32_t> list;
    for (size_t i = 0; i < c->touch.size(); ++i)
      if (c->touch[i].cls != 1) list.push_back((int32_t)i);
    const size_t n0 = list.size();
    for (size_t i = 0; i < c->touch.size(); ++i)
      if (c->touch[i].cls == 1 && c->touch[i].l < c->touch[i].m) list.push_back(~(int32_t)i);
    c->n_touch_list = (int64_t)list.size();
    c->n_touch_sym = (int64_t)(list.size() - n0);
    if (!list.empty() &&
        (rc = upload(c, (void **)&c->d_touch_list, list.data(), list.size() * sizeof(int32_t))))
      return rc;
  }
  // separated pairs, unordered, each once: test row l takes the next np(l) panels l+1, l+2, ...
  // modulo E_x (round-robin pairing: with E_x odd every row has (E_x-1)/2 partners, with E_x even
  // the rows l < E_x/2 have E_x/2 and the others E_x/2 - 1), so that all rows carry the same
  // number of full 64-lane waves instead of a ragged last wave per row; one wave per 64 partners
  {
    std::vector<int32_t> tasks;
    const int64_t n = (int64_t)ne, half = n / 2;
    for (int64_t l = 0; l < n; ++l) {
      const int64_t np = (n % 2 == 0 && l >= half) ? half - 1 : half;  // n odd: half = (n-1)/2
      for (int64_t c0 = 0; c0 < np; c0 += 64) {
        tasks.push_back((int32_t)l);
        tasks.push_back((int32_t)((l + 1 + c0) % n));
        tasks.push_back((int32_t)std::min<int64_t>(64, np - c0));
      }
    }
    c->n_sep_tasks = (int64_t)tasks.size() / 3;
    if (!tasks.empty())
      if ((rc = upload(c, (void **)&c->d_sep_tasks, tasks.data(), tasks.size() * sizeof(int32_t))))
        return rc;
    // the distinct vertices of each task's trial panels (slots, in order of first appearance) and
    // each lane's slot of its trial panel's three vertices: the kernel gathers the test row's
    // double-layer contributions per vertex in LDS and adds each vertex once per pass
    std::vector<int32_t> vstart(1, 0), verts;
    std::vector<uint8_t> slots((size_t)c->n_sep_tasks * 3 * 64, 0);
    std::unordered_map<int32_t, int> slot_of;
    for (int64_t t = 0; t < c->n_sep_tasks; ++t) {
      slot_of.clear();
      const int64_t m0 = tasks[3 * t + 1], cnt = tasks[3 * t + 2];
      for (int64_t i = 0; i < cnt; ++i) {
        const int64_t m = (m0 + i) % n;
        for (int k = 0; k < 3; ++k) {
          const int32_t v = c->tris[3 * m + k];
          auto it = slot_of.find(v);
          int sidx;
          if (it == slot_of.end()) {
            sidx = (int)slot_of.size();
            slot_of.emplace(v, sidx);
            verts.push_back(v);
          } else {
            sidx = it->second;
          }
          slots[((size_t)t * 3 + k) * 64 + i] = (uint8_t)sidx;  // at most 3 * 64 = 192 slots
        }
      }
      vstart.push_back((int32_t)verts.size());
    }
    if (!tasks.empty()) {
      if ((rc = upload(c, (void **)&c->d_sep_vstart, vstart.data(), vstart.size() * sizeof(int32_t)))) return rc;
      if ((rc = upload(c, (void **)&c->d_sep_verts, verts.data(), verts.size() * sizeof(int32_t)))) return rc;
      if ((rc = upload(c, (void **)&c->d_sep_slots, slots.data(), slots.size()))) return rc;
    }
  }
  // preconditioner pattern: itself, edge neighbours, vertex neighbours by centroid distance
  {
    std::vector<double> cent(3 * ne);
    for (size_t t = 0; t < ne; ++t)
      for (int k = 0; k < 3; ++k)
        cent[3 * t + k] = (c->verts[3 * c->tris[3 * t] + k] + c->verts[3 * c->tris[3 * t + 1] + k] +
                           c->verts[3 * c->tris[3 * t + 2] + k]) / 3.0;
    std::vector<std::vector<std::pair<double, int>>> nb(ne);
    std::vector<std::vector<int8_t>> nbc(ne);
    for (const auto &tp : c->touch) {
      double d2 = 0;
      for (int k = 0; k < 3; ++k) d2 += (cent[3 * tp.l + k] - cent[3 * tp.m + k]) * (cent[3 * tp.l + k] - cent[3 * tp.m + k]);
      // sort key: class first (3, 2, 1), then distance
      nb[tp.l].push_back({(3 - tp.cls) * 1e30 + d2, tp.m});
    }
    std::vector<int32_t> cols(ne * HB_PC_SLOTS, -1);
    std::vector<int8_t> clsv(ne * HB_PC_SLOTS, 0);
    for (size_t l = 0; l < ne; ++l) {
      std::sort(nb[l].begin(), nb[l].end());
      for (size_t s2 = 0; s2 < nb[l].size() && s2 < (size_t)HB_PC_SLOTS; ++s2) {
        cols[l * HB_PC_SLOTS + s2] = nb[l][s2].second;
        clsv[l * HB_PC_SLOTS + s2] = (int8_t)(3 - (int)(nb[l][s2].first / 1e30));
      }
    }
    if ((rc = upload(c, (void **)&c->d_pc_cols, cols.data(), cols.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, (void **)&c->d_pc_cls, clsv.data(), clsv.size()))) return rc;
    if ((rc = upload(c, (void **)&c->d_cent, cent.data(), cent.size() * sizeof(double)))) return rc;
  }
  // hypersingular operator: odd Taylor tables of D^{2,d} (d >= kD2Closed), their scales, the
  // surface curls of the local p1 basis and the vertex -> (panel, local index) lists
  {
    // degrees from the truncation bound (dropped terms below ~1.5e-15 of the block scale,
    // e^{-w}-weighted over w in [0, 128]); their changes fall on even d, so the blocks of a pass
    // (kD2Closed + 2k, kD2Closed + 2k + 1) share one length
    auto d2deg = [](int d) {
      return d < 6 ? 22 : d < 8 ? 18 : d < 12 ? 14 : d < 16 ? 12 : d < 32 ? 10 : d < 64 ? 8 : 6;
    };
    std::vector<double> d2tab((size_t)c->nt * kTaylorND, 0.0), d2sc(c->nt, 0.0);
    // per pass the shortest prefix for the pairs' distance bound, as for V_h and K_h above
    std::vector<int32_t> d2len((size_t)c->nt * 2, 0);
    for (int d = kD2Closed; d < c->nt; ++d) {
      ld poly[kTaylorND];
      const int deg = d2deg(d);
      taylor_poly_odd(d, deg, poly, kTaylorND);
      const int ps = d - ((d - kD2Closed) & 1);
      const ld cd = 1.0L / (4.0L * al * d * h);
      for (int t = 0; t < 2; ++t) {
        int32_t &L = d2len[2 * ps + t];
        L = std::max<int32_t>(L, taylor_len(poly, deg + 2, (t ? rho2_touch : rho2_sep) * cd, 1e-16L));
      }
      for (int j = 0; j < kTaylorND; ++j) d2tab[(size_t)d * kTaylorND + j] = (double)poly[j];
      d2sc[d] = (double)(al * h * powl(4.0L * kPi * al * d * h, -1.5L));
    }
    if ((rc = upload(c, (void **)&c->d_d2tab, d2tab.data(), d2tab.size() * sizeof(double)))) return rc;
    if ((rc = upload(c, (void **)&c->d_d2scale, d2sc.data(), d2sc.size() * sizeof(double)))) return rc;
    for (int d = kD2Closed; d < c->nt; ++d)
      for (int t = 0; t < 2; ++t) {
        int32_t &L = d2len[2 * d + t];
        if (L == 0) continue;
        const int full = d2deg(d) + 2;
        for (int n : kD2Lens)
          if (n >= L) { L = n; break; }
        L = std::min(L, full);
      }
    if ((rc = upload(c, (void **)&c->d_d2len, d2len.data(), d2len.size() * sizeof(int32_t)))) return rc;
    const size_t ne_ = c->ne;
    std::vector<double> curl(9 * ne_);
    for (size_t t = 0; t < ne_; ++t) {
      const double *x[3] = {&c->verts[3 * c->tris[3 * t]], &c->verts[3 * c->tris[3 * t + 1]],
                            &c->verts[3 * c->tris[3 * t + 2]]};
      for (int k = 0; k < 3; ++k)  // curl of lambda_k = n x grad lambda_k = (x_{k+1} - x_{k+2}) / (2 area)
        for (int q = 0; q < 3; ++q)
          curl[9 * t + 3 * k + q] = (x[(k + 1) % 3][q] - x[(k + 2) % 3][q]) / (2.0 * c->area[t]);
    }
    if ((rc = upload(c, (void **)&c->d_curl, curl.data(), curl.size() * sizeof(double)))) return rc;
    Adjacency A = vertex_triangles(c->tris.data(), c->nv, c->ne);
    std::vector<int32_t> vstart(c->nv + 1), vadj(6 * ne_);
    for (int64_t i = 0; i <= c->nv; ++i) vstart[i] = (int32_t)A.start[i];
    for (int64_t i = 0; i < c->nv; ++i)
      for (int64_t e = A.start[i]; e < A.start[i + 1]; ++e) {
        const int32_t t = A.tri[e];
        int k = 0;
        while (c->tris[3 * t + k] != (int32_t)i) ++k;
        vadj[2 * e] = t;
        vadj[2 * e + 1] = k;
      }
    if ((rc = upload(c, (void **)&c->d_vstart, vstart.data(), vstart.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, (void **)&c->d_vadj, vadj.data(), vadj.size() * sizeof(int32_t)))) return rc;
  }
  // regularised rules
  for (int cls = 1; cls <= 3; ++cls) {
    std::vector<SSNode> nodes;
    ss_nodes(cls, c->opt.ss_order, nodes);
    int n = (int)nodes.size(), np = (n + 63) / 64 * 64;
    std::vector<double> tab(11 * (size_t)np, 0.0);
    for (int i = 0; i < np; ++i) {
      bool real = i < n;
      for (int k = 0; k < 4; ++k) tab[(size_t)k * np + i] = real ? (double)nodes[i].c[k] : (k == 0 ? 1.0 : 0.0);
      tab[(size_t)4 * np + i] = real ? (double)nodes[i].w : 0.0;
      for (int k = 0; k < 3; ++k) tab[(size_t)(5 + k) * np + i] = real ? (double)nodes[i].lam[k] : 0.0;
      for (int k = 0; k < 3; ++k) tab[(size_t)(8 + k) * np + i] = real ? (double)nodes[i].lamx[k] : 0.0;
    }
    c->ss[cls].n = np;
    if ((rc = upload(c, (void **)&c->ss[cls].d, tab.data(), tab.size() * sizeof(double)))) return rc;
  }
  p.taylor = c->d_taylor;
  p.taylor32 = c->d_taylor32;
  p.tdeg = c->d_tdeg;
  p.tlen_sep = c->d_tlen_sep;
  p.tlen_touch = c->d_tlen_touch;
  p.tscale = c->d_tscale;
  p.geom = c->d_geom;
  p.tris = c->d_tris;
  return HB_OK;
}

// ---------------------------------------------------------------------------------------------
// Non-uniform time grid (the outlook of Sec. 7; block integrals of Sec. 3.1 / 3.2 at general
// interval endpoints).  Block (k, i), i < k, is the integral of w(s) G(rho, s) over the support
// [s1, s4] = [t_k - t_{i+1}, t_{k+1} - t_i], w the trapezoid (convolution of the indicators of
// the two intervals, widths a = h_k and b = h_i, mass a b, symmetric about c = (s1 + s4) / 2).
// Taylor form: with f(s) = s^{-p} e^{-rho^2/(4 alpha s)} and f^{(n)}(c) = c^{-p-n} e^{-w} Q_n(w)
// (the uniform tables' Q_n), the odd moments of w vanish and
//   block = (a b) c^{-p} e^{-w} sum_j m_j c^{-2j} Q_{2j}(w) / (2j)!,
//   m_j = E[(X + Y)^{2j}],  X ~ U(-a/2, a/2), Y ~ U(-b/2, b/2).
// The series converges for s1 > 0 like ((s4 - s1) / (s4 + s1))^{2j}.  Its truncation is bounded
// by sum_{j > J} |m_j c^{-2j} / (2j)!| max_{0 <= w <= 128} |Q_{2j}(w)| e^{-w} (no cancellation
// assumed); a block takes the Taylor form when this bound is below 2e-16 of its scale at some
// degree 2J <= 28 (for V and K), else the closed four-term difference.
// ---------------------------------------------------------------------------------------------
constexpr int kNuJ = 24;  // terms kept for the truncation bound (degree 48)

struct NuBounds {
  std::vector<ld> Q[2][2 * kNuJ + 1];  // Q_n coefficients, p = 3/2 (V) and 5/2 (K)
  ld M[2][2 * kNuJ + 1];               // max over the samples of |Q_n(w)| e^{-w}
};

const NuBounds &nu_bounds() {
  static NuBounds B;
  static bool ready = false;
  if (ready) return B;
  std::vector<ld> ws;
  for (int i = 0; i <= 80; ++i) ws.push_back(0.05L * i);
  for (int i = 1; i <= 248; ++i) ws.push_back(4.0L + 0.5L * i);
  for (int v = 0; v < 2; ++v) {
    const ld p = v == 0 ? 1.5L : 2.5L;
    B.Q[v][0] = {1.0L};
    for (int n = 0; n < 2 * kNuJ; ++n) {
      const auto &q = B.Q[v][n];
      std::vector<ld> r(q.size() + 1, 0.0L);
      for (size_t j = 0; j < q.size(); ++j) {
        r[j + 1] += q[j];
        r[j] -= (n + p) * q[j];
        r[j] -= (ld)j * q[j];
      }
      B.Q[v][n + 1] = r;
    }
    for (int n = 0; n <= 2 * kNuJ; ++n) {
      ld mx = 0.0L;
      for (ld w : ws) {
        ld acc = 0.0L;
        for (size_t j = B.Q[v][n].size(); j-- > 0;) acc = acc * w + B.Q[v][n][j];
        mx = std::max(mx, fabsl(acc) * expl(-w));
      }
      B.M[v][n] = mx;
    }
  }
  ready = true;
  return B;
}

// m_j c^{-2j} / (2j)! for j = 0 .. kNuJ
void nu_series_factors(ld a, ld b, ld c, ld out[kNuJ + 1]) {
  ld ma[2 * kNuJ + 1], mb[2 * kNuJ + 1];  // E[X^n], E[Y^n] (even n)
  for (int n = 0; n <= 2 * kNuJ; n += 2) {
    ma[n] = powl(a / 2, n) / (n + 1);
    mb[n] = powl(b / 2, n) / (n + 1);
  }
  ld fact = 1.0L;  // (2j)!
  for (int j = 0; j <= kNuJ; ++j) {
    if (j > 0) fact *= (ld)(2 * j - 1) * (ld)(2 * j);
    ld m = 0.0L, binom = 1.0L;  // C(2j, 2q)
    for (int q = 0; q <= j; ++q) {
      m += binom * ma[2 * q] * mb[2 * (j - q)];
      binom *= (ld)(2 * j - 2 * q) * (ld)(2 * j - 2 * q - 1) / ((ld)(2 * q + 1) * (ld)(2 * q + 2));
    }
    out[j] = m * powl(c, -2 * j) / fact;
  }
}

// Smallest tabulated degree (6, 8, ..., 20, 24, 28) whose truncation bound is below tol for V and
// K, or -1.
int nu_taylor_degree(const ld f[kNuJ + 1]) {
  static const int degs[] = {6, 8, 10, 12, 14, 16, 18, 20, 24, 28};
  const NuBounds &B = nu_bounds();
  for (int deg : degs) {
    bool ok = true;
    for (int v = 0; v < 2 && ok; ++v) {
      ld tail = 0.0L;
      for (int j = deg / 2 + 1; j <= kNuJ; ++j) tail += fabsl(f[j]) * B.M[v][2 * j];
      ok = tail <= 2e-16L * f[0];
    }
    if (ok) return deg;
  }
  return -1;
}

void nu_level(ld al, ld delta, hb::NuClosed &cb, int j, double sg) {
  const ld sq = sqrtl(al * delta);
  cb.c[j] = delta > 0 ? (double)(1.0L / (2.0L * sq)) : 0.0;
  cb.s2[j] = (double)(2.0L * al * delta);
  cb.s1[j] = (double)(2.0L * sq / sqrtl(kPi));
  cb.t2[j] = (double)(4.0L * sq / sqrtl(kPi));
  cb.sg[j] = sg;
}

int build_nu_tables(hb_ctx *c) {
  using namespace hb;
  const int nt = c->nt;
  const ld al = c->alpha;
  const std::vector<double> &t = c->tnodes;
  std::vector<NuClosed> closed;
  struct TEntry {
    int32_t out, deg;
    ld a, b, cc;
  };
  std::vector<TEntry> tay;
  for (int k = 0; k < nt; ++k)
    for (int i = 0; i <= k; ++i) {
      const int32_t out = k * (k + 1) / 2 + i;
      const ld hk = (ld)t[k + 1] - (ld)t[k], hi = (ld)t[i + 1] - (ld)t[i];
      if (i == k) {  // h_k G^{dtau}(rho, 0) + F(0) - F(h_k)
        NuClosed cb{};
        cb.out = out;
        cb.diag = 1;
        cb.nlev = 2;
        nu_level(al, 0.0L, cb, 0, 1.0);
        nu_level(al, hk, cb, 1, -1.0);
        cb.kVs = (double)(hk / (4.0L * kPi * al));
        cb.kKs = (double)(hk / (4.0L * kPi));
        closed.push_back(cb);
        continue;
      }
      const ld s1 = (ld)t[k] - (ld)t[i + 1], s4 = (ld)t[k + 1] - (ld)t[i];
      if (s1 > 0) {
        ld f[kNuJ + 1];
        const ld cc = 0.5L * (s1 + s4);
        nu_series_factors(hk, hi, cc, f);
        const int deg = nu_taylor_degree(f);
        if (deg > 0) {
          tay.push_back({out, deg, hk, hi, cc});
          continue;
        }
      }
      // F(t_k - t_i) + F(t_{k+1} - t_{i+1}) - F(t_{k+1} - t_i) - F(t_k - t_{i+1})
      NuClosed cb{};
      cb.out = out;
      cb.diag = 0;
      cb.nlev = 4;
      nu_level(al, (ld)t[k] - (ld)t[i], cb, 0, 1.0);
      nu_level(al, (ld)t[k + 1] - (ld)t[i + 1], cb, 1, 1.0);
      nu_level(al, s4, cb, 2, -1.0);
      nu_level(al, std::max(s1, 0.0L), cb, 3, -1.0);
      closed.push_back(cb);
    }
  // Taylor entries by falling degree (stable), in pairs that share the first entry's length
  std::stable_sort(tay.begin(), tay.end(), [](const TEntry &x, const TEntry &y) { return x.deg > y.deg; });
  const size_t nT = tay.size();
  std::vector<double> tab(nT * 2 * kTaylorN, 0.0), tsc(nT * 3, 0.0);
  std::vector<int32_t> tdeg(nT * 2, 0), tout(nT, 0);
  const NuBounds &B = nu_bounds();
  for (size_t b = 0; b < nT; ++b) {
    const TEntry &e = tay[b];
    const int deg = tay[b - (b & 1)].deg;  // the pass takes the first entry's length
    ld f[kNuJ + 1];
    nu_series_factors(e.a, e.b, e.cc, f);
    for (int v = 0; v < 2; ++v) {
      ld poly[kTaylorN];
      for (int j = 0; j < kTaylorN; ++j) poly[j] = 0.0L;
      for (int j = 0; j <= deg / 2; ++j)
        for (size_t q = 0; q < B.Q[v][2 * j].size() && (int)q < kTaylorN; ++q) poly[q] += f[j] * B.Q[v][2 * j][q];
      // normalised so that the scale below carries the mass a b (f[0] = 1)
      for (int j = 0; j < kTaylorN; ++j) tab[(b * 2 + v) * kTaylorN + j] = (double)poly[j];
      // the pass's lengths for the two pair classes' distance bounds, as on uniform grids (the
      // double layer takes P - P' of the single layer's polynomial, v = 0)
      if (v == 0) {
        const ld cw = 1.0L / (4.0L * al * e.cc);
        const size_t b0 = b - (b & 1);
        tdeg[2 * b0] = std::max<int32_t>(tdeg[2 * b0], taylor_len(poly, deg + 1, (ld)c->rho2_sep * cw, 1e-16L));
        tdeg[2 * b0 + 1] =
            std::max<int32_t>(tdeg[2 * b0 + 1], taylor_len(poly, deg + 1, (ld)c->rho2_touch * cw, 1e-16L));
      }
    }
    const ld mu0 = e.a * e.b;
    tsc[3 * b + 0] = (double)(mu0 * powl(4.0L * kPi * al * e.cc, -1.5L));
    tsc[3 * b + 1] = (double)(mu0 / (16.0L * powl(kPi * al, 1.5L) * powl(e.cc, 2.5L)));
    tsc[3 * b + 2] = (double)(1.0L / (4.0L * al * e.cc));
    tout[b] = e.out;
  }
  // round each pass's lengths up to an instantiated one (never past the first entry's degree + 1)
  // and give both entries of the pass the same values
  for (size_t b = 0; b < nT; b += 2)
    for (int t = 0; t < 2; ++t) {
      int32_t L = tdeg[2 * b + t];
      for (int n : kPolyLens)
        if (n >= L) { L = n; break; }
      L = std::min<int32_t>(L, tay[b].deg + 1);
      tdeg[2 * b + t] = L;
      if (b + 1 < nT) tdeg[2 * (b + 1) + t] = L;
    }
  std::vector<double> hs(nt);
  for (int k = 0; k < nt; ++k) hs[k] = t[k + 1] - t[k];
  int rc;
  if ((rc = upload(c, (void **)&c->d_nu_closed, closed.data(), closed.size() * sizeof(NuClosed)))) return rc;
  if (nT > 0) {
    if ((rc = upload(c, (void **)&c->d_nu_taylor, tab.data(), tab.size() * sizeof(double)))) return rc;
    if ((rc = upload(c, (void **)&c->d_nu_tscale, tsc.data(), tsc.size() * sizeof(double)))) return rc;
    if ((rc = upload(c, (void **)&c->d_nu_tdeg, tdeg.data(), tdeg.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(c, (void **)&c->d_nu_tout, tout.data(), tout.size() * sizeof(int32_t)))) return rc;
  }
  if ((rc = upload(c, (void **)&c->d_nu_h, hs.data(), hs.size() * sizeof(double)))) return rc;
  if ((rc = upload(c, (void **)&c->d_nu_t, c->tnodes.data(), c->tnodes.size() * sizeof(double))))
    return rc;
  c->n_nu_closed = (int32_t)closed.size();
  c->n_nu_taylor = (int32_t)nT;
  return HB_OK;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

void hb_default_options(hb_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->ss_order = 4;
  o->d_switch = 3;
  o->storage = HB_DTYPE_F64;
  o->mixed_d_min = 3;
}

int hb_check_mesh(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                  int64_t class_counts[4]) {
  int rc = validate_mesh(nullptr, verts, n_verts, tris, n_tris);
  if (rc) return rc;
  if (class_counts) count_classes(tris, n_verts, n_tris, class_counts, nullptr, nullptr);
  return HB_OK;
}

const char *hb_last_error(const hb_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

}  // extern "C"

// Context creation shared by hb_create (uniform steps, t_nodes NULL) and hb_create_nonuniform.
static int create_ctx(hb_ctx **out, const double *verts, int64_t n_verts, const int32_t *tris,
                      int64_t n_tris, double alpha, double T, int32_t n_t, const hb_options *opt,
                      const double *t_nodes) {
  if (!out) return fail(nullptr, HB_EINVAL, "out is null");
  *out = nullptr;
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(nullptr, HB_EINVAL, "alpha must be > 0");
  if (t_nodes) {
    if (n_t < 1 || n_t > 4096) return fail(nullptr, HB_EINVAL, "n_t must be in 1..4096 on a non-uniform grid");
    if (t_nodes[0] != 0.0) return fail(nullptr, HB_EINVAL, "t_nodes[0] must be 0");
    for (int k = 0; k < n_t; ++k)
      if (!(t_nodes[k + 1] > t_nodes[k]) || !std::isfinite(t_nodes[k + 1]))
        return fail(nullptr, HB_EINVAL, "t_nodes must be finite and strictly increasing");
    T = t_nodes[n_t];
  }
  if (!(T > 0) || !std::isfinite(T)) return fail(nullptr, HB_EINVAL, "T must be > 0");
  if (n_t < 1 || n_t > 65536) return fail(nullptr, HB_EINVAL, "n_t must be in 1..65536");
  hb_options o;
  hb_default_options(&o);
  if (opt) o = *opt;
  if (o.ss_order < 1 || o.ss_order > 8) return fail(nullptr, HB_EINVAL, "ss_order must be in 1..8");
  if (o.d_switch != 3 && o.d_switch != 8 && o.d_switch != 16)
    return fail(nullptr, HB_EINVAL, "d_switch must be 3, 8 or 16");
  if (o.storage != HB_DTYPE_F64 && o.storage != HB_DTYPE_F32)
    return fail(nullptr, HB_EINVAL, "storage must be HB_DTYPE_F64 or HB_DTYPE_F32");
  if (o.mixed_d_min < 2) return fail(nullptr, HB_EINVAL, "mixed_d_min must be >= 2");
  for (int i = 0; i < 12; ++i)
    if (o.reserved[i]) return fail(nullptr, HB_EINVAL, "reserved options must be zero");
  if (t_nodes && o.storage != HB_DTYPE_F64)
    return fail(nullptr, HB_EINVAL, "a non-uniform grid needs HB_DTYPE_F64 storage");
  int rc = validate_mesh(nullptr, verts, n_verts, tris, n_tris);
  if (rc) return rc;
  hb_ctx *c = new hb_ctx();
  c->ne = n_tris;
  c->nv = n_verts;
  c->nt = n_t;
  c->nb = n_t;
  if (t_nodes) {
    c->nu = true;
    c->tnodes.assign(t_nodes, t_nodes + n_t + 1);
    c->nb = (int64_t)n_t * (n_t + 1) / 2;
  }
  c->alpha = alpha;
  c->T = T;
  c->h = T / n_t;
  c->opt = o;
  c->storage_f32 = o.storage == HB_DTYPE_F32;
  c->verts.assign(verts, verts + 3 * n_verts);
  c->tris.assign(tris, tris + 3 * n_tris);
  count_classes(tris, n_verts, n_tris, c->n_class, &c->touch, verts);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, HB_EHIP, "no HIP device");
  }
  rc = build_tables(c);
  if (!rc && c->nu) rc = build_nu_tables(c);
  if (!rc) rc = hb::static_scratch_init(c);
  if (rc) {
    g_err = c->err;
    hb_destroy(c);
    return rc;
  }
  for (int i = 0; i < 4; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) {
      hb_destroy(c);
      return fail(nullptr, HB_EHIP, "hipEventCreate failed");
    }
  *out = c;
  return HB_OK;
}

extern "C" {

int hb_create(hb_ctx **out, const double *verts, int64_t n_verts, const int32_t *tris,
              int64_t n_tris, double alpha, double T, int32_t n_t, const hb_options *opt) {
  return create_ctx(out, verts, n_verts, tris, n_tris, alpha, T, n_t, opt, nullptr);
}

int hb_create_nonuniform(hb_ctx **out, const double *verts, int64_t n_verts, const int32_t *tris,
                         int64_t n_tris, double alpha, const double *t_nodes, int32_t n_t,
                         const hb_options *opt) {
  if (!t_nodes) return fail(nullptr, HB_EINVAL, "t_nodes is null");
  return create_ctx(out, verts, n_verts, tris, n_tris, alpha, 0.0, n_t, opt, t_nodes);
}

int hb_is_nonuniform(const hb_ctx *c) { return c && c->nu ? 1 : 0; }

void hb_destroy(hb_ctx *c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  void *ptrs[] = {c->d_params, c->d_params_repr, c->d_geom, c->d_tris, c->d_touch, c->d_touch_list, c->d_sep_tasks, c->d_sep_vstart, c->d_sep_verts, c->d_sep_slots, c->d_taylor,
                  c->d_taylor32, c->d_tdeg, c->d_tlen_sep, c->d_tlen_touch, c->d_V32, c->d_tscale, c->d_mass,
                  c->d_V, c->d_K, c->d_KT, c->d_work, c->d_v0inv, c->d_apply, c->d_ir,
                  c->d_pc_cols, c->d_pc_cls, c->d_cent, c->d_pc_M, c->d_reprq, c->ss[1].d, c->ss[2].d, c->ss[3].d,
                  c->d_D, c->d_Dw, c->d_V11, c->d_minv, c->d_pcw, c->d_Kt, c->d_near_sep, c->d_near_touch, c->d_d2tab, c->d_d2scale, c->d_d2len, c->d_curl, c->d_vstart,
                  c->d_vadj, c->d_pc_buf, c->d_nu_closed, c->d_nu_tout, c->d_nu_tdeg, c->d_nu_taylor,
                  c->d_nu_tscale, c->d_nu_h, c->d_nu_t};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (int i = 0; i < 4; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->ev_step) (void)hipEventDestroy(c->ev_step);
  if (c->ev_prev) (void)hipEventDestroy(c->ev_prev);
  if (c->h_res) (void)hipHostFree(c->h_res);
  delete c;
}

int hb_sizes(const hb_ctx *c, int64_t *ne, int64_t *nv, int32_t *nt, int64_t *ntouch) {
  if (!c) return fail(nullptr, HB_EINVAL, "null context");
  if (ne) *ne = c->ne;
  if (nv) *nv = c->nv;
  if (nt) *nt = c->nt;
  if (ntouch) *ntouch = (int64_t)c->touch.size();
  return HB_OK;
}

// The p1 x p1 operators: V_h^{11} (Sec. 6.1) and D_h (Sec. 3.3, from the assembled V_h); the kernels
// read the parameters of the last assembly (uploaded here if none has run).
static int assemble_p1(hb_ctx *c, uint32_t ops, hipStream_t s) {
  const size_t nD = (size_t)c->nt * c->nv * c->nv, esz = c->storage_f32 ? 4 : 8;
  if (!c->d_params) {
    c->launch = c->params;
    c->launch.V = c->d_V;
    HB_HIP(c, hipMalloc(&c->d_params, sizeof(hb::AsmParams)));
    HB_HIP(c, hipMemcpyAsync(c->d_params, &c->launch, sizeof(c->launch), hipMemcpyHostToDevice, s));
  }
  if (!c->d_Dw) HB_HIP(c, hipMalloc(&c->d_Dw, nD * esz));
  if (ops & HB_OP_V11) {
    if (!c->d_V11) {
      HB_HIP(c, hipMalloc(&c->d_V11, nD * esz + hb::kBlockPad));
      HB_HIP(c, hipMemsetAsync((char *)c->d_V11 + nD * esz, 0, hb::kBlockPad, s));
    }
    int rc = hb::launch_assemble_v11(c, s);
    if (rc) return fail(c, rc, "V11 assembly launch failed");
    c->have_V11 = true;
  }
  if (ops & HB_OP_D) {
    if (!c->d_D) {
      HB_HIP(c, hipMalloc(&c->d_D, nD * esz + hb::kBlockPad));
      HB_HIP(c, hipMemsetAsync((char *)c->d_D + nD * esz, 0, hb::kBlockPad, s));
    }
    int rc = hb::launch_assemble_d(c, s);
    if (rc) return fail(c, rc, "hypersingular assembly launch failed");
    c->have_D = true;
  }
  return HB_OK;
}

// Assembly on a non-uniform grid: V^{k,i}, K^{k,i} for all 0 <= i <= k < E_t (packed), FP64.
static int assemble_nu(hb_ctx *c, uint32_t ops, int32_t precision, hipStream_t s) {
  if (ops & ~(HB_OP_V | HB_OP_K))
    return fail(c, HB_EINVAL, "a non-uniform grid has HB_OP_V and HB_OP_K only");
  if (precision != HB_PREC_FP64) return fail(c, HB_EINVAL, "a non-uniform grid is assembled in FP64 only");
  const size_t nV = (size_t)c->nb * c->ne * c->ne, nK = (size_t)c->nb * c->ne * c->nv, esz = 8;
  if ((ops & HB_OP_V) && !c->d_V) {
    HB_HIP(c, hipMalloc(&c->d_V, nV * esz + hb::kBlockPad));
    HB_HIP(c, hipMemsetAsync((char *)c->d_V + nV * esz, 0, hb::kBlockPad, s));
  }
  if ((ops & HB_OP_K) && !c->d_K) {
    HB_HIP(c, hipMalloc(&c->d_K, nK * esz + hb::kBlockPad));
    HB_HIP(c, hipMemsetAsync((char *)c->d_K + nK * esz, 0, hb::kBlockPad, s));
  }
  if ((ops & HB_OP_K) && !c->d_KT) HB_HIP(c, hipMalloc(&c->d_KT, nK * esz));
  hb::AsmParams &p = c->launch;
  p = c->params;
  p.V = c->d_V;
  p.K = c->d_K;
  p.KT = c->d_KT;
  p.do_V = (ops & HB_OP_V) ? 1 : 0;
  p.do_K = (ops & HB_OP_K) ? 1 : 0;
  if (!c->d_params) HB_HIP(c, hipMalloc(&c->d_params, sizeof(hb::AsmParams)));
  HB_HIP(c, hipMemcpyAsync(c->d_params, &p, sizeof(p), hipMemcpyHostToDevice, s));
  if (p.do_K) {
    HB_HIP(c, hipMemsetAsync(c->d_K, 0, nK * esz, s));
    HB_HIP(c, hipMemsetAsync(c->d_KT, 0, nK * esz, s));
  }
  hb::NuTabs nu{c->d_nu_closed, c->n_nu_closed, c->n_nu_taylor, c->d_nu_tout, c->d_nu_taylor,
                c->d_nu_tscale, c->d_nu_tdeg};
  HB_HIP(c, hipEventRecord(c->ev[0], s));
  if (c->n_sep_tasks > 0) hb::launch_nu_separated(c->d_params, nu, c->d_sep_tasks, c->n_sep_tasks, s);
  HB_HIP(c, hipGetLastError());
  if (p.do_K) {
    hb::AsmParams fold = p;  // the fold runs over the nb packed blocks
    fold.nt = (int32_t)c->nb;
    hb::launch_fold_KT(fold, 0, s);
    HB_HIP(c, hipGetLastError());
  }
  HB_HIP(c, hipEventRecord(c->ev[1], s));
  const int64_t ntouch = c->n_class[1] + c->n_class[2] + c->n_class[3];
  if (ntouch > 0) hb::launch_nu_touching(c->d_params, nu, c->d_touch, ntouch, c->ss, s);
  HB_HIP(c, hipGetLastError());
  HB_HIP(c, hipEventRecord(c->ev[2], s));
  if (p.do_V) {
    c->have_V = true;
    c->v0inv_valid = false;  // the inverses of the diagonal blocks V^{k,k}
  }
  if (p.do_K) c->have_K = true;
  c->timed = true;
  return HB_OK;
}

int hb_assemble(hb_ctx *c, uint32_t ops, int32_t precision, void *stream) {
  if (!c) return fail(nullptr, HB_EINVAL, "null context");
  if (c->nu) {
    if (ops == 0) return fail(c, HB_EINVAL, "ops must be a non-empty subset of HB_OP_V | HB_OP_K");
    return assemble_nu(c, ops, precision, (hipStream_t)stream);
  }
  if (ops == 0 || (ops & ~(HB_OP_V | HB_OP_K | HB_OP_D | HB_OP_V11)))
    return fail(c, HB_EINVAL, "ops must be a non-empty subset of HB_OP_V | HB_OP_K | HB_OP_D | HB_OP_V11");
  if (precision != HB_PREC_FP64 && precision != HB_PREC_MIXED) return fail(c, HB_EINVAL, "unknown precision");
  if ((ops & HB_OP_D) && !(ops & HB_OP_V) && !c->have_V)
    return fail(c, HB_ESTATE, "HB_OP_D needs V (assembled before or in the same call)");
  hipStream_t s = (hipStream_t)stream;
  if (!(ops & (HB_OP_V | HB_OP_K))) return assemble_p1(c, ops, s);
  size_t esz = c->storage_f32 ? 4 : 8;
  size_t nV = (size_t)c->nt * c->ne * c->ne, nK = (size_t)c->nt * c->ne * c->nv;
  if ((ops & HB_OP_V) && !c->d_V) {
    HB_HIP(c, hipMalloc(&c->d_V, nV * esz + hb::kBlockPad));
    HB_HIP(c, hipMemsetAsync((char *)c->d_V + nV * esz, 0, hb::kBlockPad, s));
  }
  if ((ops & HB_OP_K) && !c->d_K) {
    HB_HIP(c, hipMalloc(&c->d_K, nK * esz + hb::kBlockPad));
    HB_HIP(c, hipMemsetAsync((char *)c->d_K + nK * esz, 0, hb::kBlockPad, s));
  }
  if ((ops & HB_OP_K) && !c->d_KT) HB_HIP(c, hipMalloc(&c->d_KT, nK * esz));
  hb::AsmParams &p = c->launch;
  p = c->params;
  p.V = c->d_V;
  p.K = c->d_K;
  p.KT = c->d_KT;
  p.do_V = (ops & HB_OP_V) ? 1 : 0;
  p.do_K = (ops & HB_OP_K) ? 1 : 0;
  p.mixed_d_min = precision == HB_PREC_MIXED ? c->opt.mixed_d_min : c->nt;
  if (!c->d_params) HB_HIP(c, hipMalloc(&c->d_params, sizeof(hb::AsmParams)));
  HB_HIP(c, hipMemcpyAsync(c->d_params, &p, sizeof(p), hipMemcpyHostToDevice, s));
  // K is accumulated over the (up to three) panels of each trial vertex: clear it first
  if (p.do_K) {
    HB_HIP(c, hipMemsetAsync(c->d_K, 0, nK * esz, s));
    HB_HIP(c, hipMemsetAsync(c->d_KT, 0, nK * esz, s));
  }
  HB_HIP(c, hipEventRecord(c->ev[0], s));
  if (c->n_sep_tasks > 0)
    hb::launch_assemble_separated(c->d_params, p, c->d_sep_tasks, c->d_sep_vstart, c->d_sep_verts,
                                  c->d_sep_slots, c->n_sep_tasks, precision,
                                  c->storage_f32, s);
  HB_HIP(c, hipGetLastError());
  if (p.do_K) {
    hb::launch_fold_KT(p, c->storage_f32, s);
    HB_HIP(c, hipGetLastError());
  }
  HB_HIP(c, hipEventRecord(c->ev[1], s));
  // all touching pairs in one launch (the list is sorted identical, edge, vertex: the longest
  // pairs start first and the classes overlap)
  if (c->n_touch_list > 0)
    hb::launch_assemble_touching(c->d_params, p, c->d_touch, c->d_touch_list, c->n_touch_list,
                                 c->n_touch_sym, c->ss, c->storage_f32, s);
  HB_HIP(c, hipGetLastError());
  HB_HIP(c, hipEventRecord(c->ev[2], s));
  if (p.do_V) {
    c->have_V = true;
    c->V32_valid = false;
    c->v0inv_valid = false;
    c->pc_active = false;  // M was scaled by the previous V^0
  }
  if (p.do_K) {
    c->have_K = true;
    c->Kt_valid = false;
  }
  c->timed = true;
  if (ops & (HB_OP_D | HB_OP_V11)) return assemble_p1(c, ops, s);
  return HB_OK;
}

int hb_last_assembly_ms(hb_ctx *c, double ms[3]) {
  if (!c || !ms) return fail(c, HB_EINVAL, "null argument");
  if (!c->timed) return fail(c, HB_ESTATE, "no assembly has run");
  HB_HIP(c, hipEventSynchronize(c->ev[2]));
  float a = 0, b = 0, t = 0;
  HB_HIP(c, hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
  HB_HIP(c, hipEventElapsedTime(&b, c->ev[1], c->ev[2]));
  HB_HIP(c, hipEventElapsedTime(&t, c->ev[0], c->ev[2]));
  ms[0] = a;
  ms[1] = b;
  ms[2] = t;
  return HB_OK;
}

int hb_nearfield_pattern(hb_ctx *c, double radius, int64_t *nnz, int64_t *row_start,
                         int32_t *cols) {
  if (!c || !nnz) return fail(c, HB_EINVAL, "null argument");
  if (c->nu) return fail(c, HB_EINVAL, "not available on a non-uniform time grid");
  if (!(radius >= 0) || !std::isfinite(radius)) return fail(c, HB_EINVAL, "radius must be finite and >= 0");
  const int64_t ne = c->ne;
  // centroids binned in cells of edge max(radius, tiny): candidates come from the 27 cells around
  std::vector<double> cent(3 * ne);
  double lo[3] = {1e300, 1e300, 1e300};
  for (int64_t t = 0; t < ne; ++t)
    for (int k = 0; k < 3; ++k) {
      cent[3 * t + k] = (c->verts[3 * c->tris[3 * t] + k] + c->verts[3 * c->tris[3 * t + 1] + k] +
                         c->verts[3 * c->tris[3 * t + 2] + k]) / 3.0;
      lo[k] = std::min(lo[k], cent[3 * t + k]);
    }
  const double cell = std::max(radius, 1e-12);
  auto key = [&](int64_t i, int64_t j, int64_t k) { return (i * 2097152 + j) * 2097152 + k; };
  std::unordered_map<int64_t, std::vector<int32_t>> grid;
  std::vector<int64_t> ci(3 * ne);
  for (int64_t t = 0; t < ne; ++t) {
    for (int k = 0; k < 3; ++k) ci[3 * t + k] = (int64_t)std::min((cent[3 * t + k] - lo[k]) / cell, 2.0e6);
    grid[key(ci[3 * t], ci[3 * t + 1], ci[3 * t + 2])].push_back((int32_t)t);
  }
  std::unordered_map<int64_t, int32_t> touch_idx;  // (l, m) -> index in the touching list
  std::vector<std::vector<int32_t>> touch_row(ne);
  for (size_t i = 0; i < c->touch.size(); ++i) {
    touch_idx[(int64_t)c->touch[i].l * ne + c->touch[i].m] = (int32_t)i;
    touch_row[c->touch[i].l].push_back(c->touch[i].m);
  }
  c->near_start.assign(ne + 1, 0);
  c->near_cols.clear();
  const double r2 = radius * radius;
  std::vector<int32_t> row;
  for (int64_t l = 0; l < ne; ++l) {
    row.clear();
    for (int64_t di = -1; di <= 1; ++di)
      for (int64_t dj = -1; dj <= 1; ++dj)
        for (int64_t dk = -1; dk <= 1; ++dk) {
          auto it = grid.find(key(ci[3 * l] + di, ci[3 * l + 1] + dj, ci[3 * l + 2] + dk));
          if (it == grid.end()) continue;
          for (int32_t m : it->second) {
            double dd = 0;
            for (int k = 0; k < 3; ++k) dd += (cent[3 * l + k] - cent[3 * m + k]) * (cent[3 * l + k] - cent[3 * m + k]);
            if (dd <= r2) row.push_back(m);
          }
        }
    row.insert(row.end(), touch_row[l].begin(), touch_row[l].end());  // every touching pair
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    c->near_cols.insert(c->near_cols.end(), row.begin(), row.end());
    c->near_start[l + 1] = (int64_t)c->near_cols.size();
  }
  const int64_t n = (int64_t)c->near_cols.size();
  std::vector<int32_t> sep, tch;
  for (int64_t l = 0; l < ne; ++l)
    for (int64_t e = c->near_start[l]; e < c->near_start[l + 1]; ++e) {
      const int32_t m = c->near_cols[e];
      auto it = touch_idx.find(l * ne + m);
      if (it == touch_idx.end()) {
        sep.push_back((int32_t)l);
        sep.push_back(m);
        sep.push_back((int32_t)e);
      } else {
        const hb::TouchPair &tp = c->touch[it->second];
        tch.push_back(it->second);
        tch.push_back((int32_t)e);
        for (int j = 0; j < 3; ++j) {
          int k = 0;
          while (c->tris[3 * m + k] != tp.vtx[j]) ++k;
          tch.push_back(k);
        }
      }
    }
  if (c->d_near_sep) (void)hipFree(c->d_near_sep);
  if (c->d_near_touch) (void)hipFree(c->d_near_touch);
  c->d_near_sep = c->d_near_touch = nullptr;
  c->near_nnz = -1;
  int rc;
  if (!sep.empty() && (rc = upload(c, (void **)&c->d_near_sep, sep.data(), sep.size() * sizeof(int32_t)))) return rc;
  if (!tch.empty() && (rc = upload(c, (void **)&c->d_near_touch, tch.data(), tch.size() * sizeof(int32_t)))) return rc;
  c->near_nsep = (int64_t)sep.size() / 3;
  c->near_ntouch = (int64_t)tch.size() / 5;
  c->near_nnz = n;
  *nnz = n;
  if (row_start) std::memcpy(row_start, c->near_start.data(), sizeof(int64_t) * (ne + 1));
  if (cols) std::memcpy(cols, c->near_cols.data(), sizeof(int32_t) * n);
  return HB_OK;
}

int hb_assemble_nearfield(hb_ctx *c, double *V, double *K, void *stream) {
  if (!c || !V || !K) return fail(c, HB_EINVAL, "null argument");
  if (c->near_nnz < 0) return fail(c, HB_ESTATE, "no near-field pattern (hb_nearfield_pattern)");
  hipStream_t s = (hipStream_t)stream;
  if (!c->d_params) {
    c->launch = c->params;
    HB_HIP(c, hipMalloc(&c->d_params, sizeof(hb::AsmParams)));
    HB_HIP(c, hipMemcpyAsync(c->d_params, &c->launch, sizeof(c->launch), hipMemcpyHostToDevice, s));
  }
  int rc = hb::launch_assemble_near(c, V, K, s);
  if (rc) return fail(c, rc, "near-field assembly launch failed");
  return HB_OK;
}

int hb_get_blocks(hb_ctx *c, uint32_t op, int32_t d0, int32_t nd, void *dst, int32_t dtype,
                  int32_t dst_on_device, void *stream) {
  if (!c || !dst) return fail(c, HB_EINVAL, "null argument");
  if (op != HB_OP_V && op != HB_OP_K && op != HB_OP_D && op != HB_OP_V11)
    return fail(c, HB_EINVAL, "op must be HB_OP_V, HB_OP_K, HB_OP_D or HB_OP_V11");
  if (d0 < 0 || nd < 0 || (int64_t)d0 + nd > c->nb) return fail(c, HB_EINVAL, "block range out of bounds");
  if (dtype != HB_DTYPE_F64 && dtype != HB_DTYPE_F32) return fail(c, HB_EINVAL, "bad dtype");
  const bool p1p1 = op == HB_OP_D || op == HB_OP_V11;
  bool have = op == HB_OP_V ? c->have_V : op == HB_OP_K ? c->have_K : op == HB_OP_D ? c->have_D : c->have_V11;
  if (!have) return fail(c, HB_ESTATE, "operator not assembled");
  const size_t rows = p1p1 ? (size_t)c->nv : (size_t)c->ne;
  size_t cols = op == HB_OP_V ? (size_t)c->ne : (size_t)c->nv;
  size_t per = rows * cols, n = per * nd;
  size_t esz = c->storage_f32 ? 4 : 8;
  const void *base = op == HB_OP_V ? c->d_V : op == HB_OP_K ? c->d_K : op == HB_OP_D ? c->d_D : c->d_V11;
  const char *src = (const char *)base + (size_t)d0 * per * esz;
  hipStream_t s = (hipStream_t)stream;
  bool same = (dtype == HB_DTYPE_F32) == (c->storage_f32 != 0);
  if (same) {
    HB_HIP(c, hipMemcpyAsync(dst, src, n * esz, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!dst_on_device) HB_HIP(c, hipStreamSynchronize(s));
    return HB_OK;
  }
  // conversion on the host
  std::vector<char> tmp(n * esz);
  HB_HIP(c, hipMemcpyAsync(tmp.data(), src, n * esz, hipMemcpyDeviceToHost, s));
  HB_HIP(c, hipStreamSynchronize(s));
  size_t osz = dtype == HB_DTYPE_F32 ? 4 : 8;
  std::vector<char> conv(n * osz);
  for (size_t i = 0; i < n; ++i) {
    if (dtype == HB_DTYPE_F32) ((float *)conv.data())[i] = (float)((const double *)tmp.data())[i];
    else ((double *)conv.data())[i] = (double)((const float *)tmp.data())[i];
  }
  if (dst_on_device) {
    HB_HIP(c, hipMemcpyAsync(dst, conv.data(), n * osz, hipMemcpyHostToDevice, s));
    HB_HIP(c, hipStreamSynchronize(s));
  } else {
    std::memcpy(dst, conv.data(), n * osz);
  }
  return HB_OK;
}

}  // extern "C"
