/*
 * oracle.c -- reference (oracle) implementation of the semi-analytic space-time Galerkin BEM for
 * the 3D heat equation (Zapletal, Watschinger, Of, Merta, arXiv 2102.09811).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain CPU checker against which the HIP
 * path is compared.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or constant generator with the HIP library.
 *
 * Precision: all method arithmetic is carried out in x87 long double (64-bit mantissa) with
 * glibc's erfl/expl/sqrtl; results are returned as double.
 *
 * What is computed, and from which passage of the paper:
 *   - heat kernel G_alpha and alpha dG/dn_y                         (Sec. 2)
 *   - temporal antiderivatives G^{dtau}, G^{dtau dt}, their normal
 *     derivatives and their limits                                  (Sec. 3.1, 3.2; summary Sec. 4)
 *   - V^d(r) (single layer, eq. for V^d and V^0) and K^d(r) (double
 *     layer, eq. for K^d and K^0) per spatial point pair            (Sec. 3.1, 3.2)
 *   - Galerkin blocks V_h^d (p0 x p0) and K_h^d (p0 test x p1 trial) with the regular
 *     triangle rule for separated pairs and Sauter-Schwab type regularised
 *     [0,1]^4 rules for touching pairs                              (Sec. 3.1 "Galerkin weights"; Sec. 5.2)
 *   - the paper's assembly order: loop over delta = i_t h, evaluate
 *     once, scatter to blocks i_t-1, i_t, i_t+1                     (Sec. 5.1, Tables 5.1/5.2, Sec. 5.2)
 *   - single- and double-layer potentials (representation formula) (Sec. 3.5)
 *   - the second part D^{2,d}(r) of the hypersingular operator and its Galerkin blocks
 *     (p1 x p1 with n(x) . n(y))                                     (Sec. 3.3, eq. for D^{2,d})
 *   - the single layer between p1 functions, V_h^{11}                (Sec. 6.1, preconditioner of D_h)
 *   - a plain double-precision assembly in the paper's level order, the timed CPU baseline
 *     (Sec. 5.1; not a parity reference)
 *   - blocks V^{k,i}_h, K^{k,i}_h on non-uniform time grids (the outlook of Sec. 7 with the block
 *     integrals of Sec. 3.1, 3.2 at general interval endpoints)
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - Small-argument series for the double-layer bracket (it cancels like 1/z^2 when
 *     z = |r|/(2 sqrt(alpha delta)) is small; the paper only gives the limit |r| -> 0).
 *   - For d > 16 the time integral of V^d / K^d is evaluated as the hat-weighted integral of
 *     G_alpha / alpha dG/dn over [(d-1)h, (d+1)h] with Gauss-Legendre nodes, which equals the
 *     closed form exactly but does not lose digits to the second difference of G^{dtau dt}.
 *   - The h G^{dtau}(r, 0) term of V^0 (and h alpha dG^{dtau}/dn(r, 0) of K^0) is added to
 *     block 0 at level i_t = 0 (the assembly sketch omits it; the block formula has it).
 *   - Touching pairs use the regularised rule at every level, separated pairs the triangle rule
 *     at every level.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

/* ------------------------------------------------------------------------------------------ */
/* Heat kernel and temporal antiderivatives (Sec. 2, Sec. 3.1, Sec. 3.2, formula summary).     */
/* ------------------------------------------------------------------------------------------ */

/* G^{dtau}_alpha(r, delta) = erf(z) / (4 pi alpha rho), z = rho / (2 sqrt(alpha delta));
 * limit delta -> 0+: 1/(4 pi alpha rho); limit rho -> 0+: 1/(4 pi^{3/2} alpha^{3/2} sqrt(delta)). */
ld or_g1(ld rho, ld delta, ld alpha) {
  if (delta <= 0.0L) return 1.0L / (4.0L * PI_L * alpha * rho);
  if (rho <= 0.0L) return 1.0L / (4.0L * powl(PI_L * alpha, 1.5L) * sqrtl(delta));
  ld z = rho / (2.0L * sqrtl(alpha * delta));
  return erfl(z) / (4.0L * PI_L * alpha * rho);
}

/* G^{dtau dt}_alpha(r, delta), with the limits delta -> 0+ (rho / (8 pi alpha^2)) and
 * rho -> 0+ (sqrt(delta) / (2 sqrt(pi^3 alpha^3))). */
ld or_F(ld rho, ld delta, ld alpha) {
  if (delta <= 0.0L) return rho / (8.0L * PI_L * alpha * alpha);
  if (rho <= 0.0L) return sqrtl(delta) / (2.0L * sqrtl(PI_L * PI_L * PI_L * alpha * alpha * alpha));
  ld z = rho / (2.0L * sqrtl(alpha * delta));
  return ((rho / (2.0L * alpha * alpha) + delta / (alpha * rho)) * erfl(z) +
          sqrtl(delta / (PI_L * alpha * alpha * alpha)) * expl(-z * z)) /
         (4.0L * PI_L);
}

/* Series of B(z) = (1 - 1/(2 z^2)) erf z + exp(-z^2)/(z sqrt(pi)) for small z:
 * B(z) = (4/sqrt(pi)) sum_n (-1)^n z^{2n+1} / (n! (2n+1)(2n+3)).  Terms are summed until they
 * drop below the long double epsilon. */
static ld bracket_B_series(ld z) {
  ld z2 = z * z, term = z, sum = 0.0L; /* term = z^{2n+1}/n! (signed) */
  for (int n = 0; n < 60; ++n) {
    ld t = term / ((ld)(2 * n + 1) * (ld)(2 * n + 3));
    sum += t;
    if (fabsl(t) < 1e-22L * fabsl(sum)) break;
    term *= -z2 / (ld)(n + 1);
  }
  return 4.0L / sqrtl(PI_L) * sum;
}

/* Series of C(z) = erf z - (2 z / sqrt(pi)) exp(-z^2) = (4/sqrt(pi)) sum_n (-1)^n z^{2n+3}/(n!(2n+3)). */
static ld bracket_C_series(ld z) {
  ld z2 = z * z, term = z * z2, sum = 0.0L;
  for (int n = 0; n < 60; ++n) {
    ld t = term / (ld)(2 * n + 3);
    sum += t;
    if (fabsl(t) < 1e-22L * fabsl(sum)) break;
    term *= -z2 / (ld)(n + 1);
  }
  return 4.0L / sqrtl(PI_L) * sum;
}

/* alpha dG^{dtau dt}/dn_y (r, delta) divided by (r . n_y).  Closed form of Sec. 3.2 for z >= 1/2,
 * the small-z series otherwise; limits delta -> 0+ (-1/(8 pi alpha rho)) and rho -> 0+ (0). */
ld or_Fn_rn(ld rho, ld delta, ld alpha) {
  if (delta <= 0.0L) return -1.0L / (8.0L * PI_L * alpha * rho);
  if (rho <= 0.0L) return 0.0L;
  ld z = rho / (2.0L * sqrtl(alpha * delta));
  if (z < 0.5L) return -bracket_B_series(z) / (8.0L * PI_L * alpha * rho);
  return -((1.0L / (2.0L * alpha) - delta / (rho * rho)) * erfl(z) +
           sqrtl(delta) / (rho * sqrtl(PI_L * alpha)) * expl(-z * z)) /
         (4.0L * PI_L * rho);
}

/* alpha dG^{dtau}/dn_y (r, delta) divided by (r . n_y); limit delta -> 0+: 1/(4 pi rho^3). */
ld or_g1n_rn(ld rho, ld delta, ld alpha) {
  if (delta <= 0.0L) return 1.0L / (4.0L * PI_L * rho * rho * rho);
  ld z = rho / (2.0L * sqrtl(alpha * delta));
  if (z < 0.5L) return bracket_C_series(z) / (4.0L * PI_L * rho * rho * rho);
  return (erfl(z) / rho - expl(-z * z) / sqrtl(PI_L * alpha * delta)) / (4.0L * PI_L * rho * rho);
}

/* ---- Gauss-Legendre nodes on [0, 1] by Newton iteration on P_n (long double) ---- */
static void gauss_legendre01(int n, ld *x, ld *w) {
  for (int i = 0; i < n; ++i) {
    ld t = cosl(PI_L * ((ld)i + 0.75L) / ((ld)n + 0.5L));
    ld dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1.0L, p1 = t;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / (ld)k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0L; }
      dp = (ld)n * (t * p1 - p0) / (t * t - 1.0L);
      ld dt = p1 / dp;
      t -= dt;
      if (fabsl(dt) < 1e-21L) break;
    }
    {
      ld p0 = 1.0L, p1 = t;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / (ld)k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0L; }
      dp = (ld)n * (t * p1 - p0) / (t * t - 1.0L);
    }
    x[i] = 0.5L * (1.0L - t);
    w[i] = 1.0L / ((1.0L - t * t) * dp * dp); /* 2/((1-t^2)P'^2) halved for [0,1] */
  }
}

/* Hat-weighted time integrals h^2 int_{-1}^{1} (1-|u|) f((d+u) h) du for f = G_alpha (out[0]) and
 * f = alpha dG/dn_y / (r . n_y) (out[1]); both share exp(-rho^2/(4 alpha s)). */
#define HAT_NT 12
static void hat_integrals(ld rho, int d, ld h, ld alpha, ld out[2]) {
  static ld gx[HAT_NT], gw[HAT_NT];
  static int ready = 0;
  if (!ready) {
#pragma omp critical(oracle_hat_init)
    {
      if (!ready) {
        gauss_legendre01(HAT_NT, gx, gw);
        __sync_synchronize();
        ready = 1;
      }
    }
  }
  const ld cG = 1.0L / ((4.0L * PI_L * alpha) * sqrtl(4.0L * PI_L * alpha)); /* (4 pi alpha)^{-3/2} */
  const ld cK = 1.0L / (16.0L * PI_L * alpha * sqrtl(PI_L * alpha));        /* 1/(16 (pi alpha)^{3/2}) */
  ld sV = 0.0L, sK = 0.0L;
  for (int i = 0; i < HAT_NT; ++i) {
    /* u in [0,1]: weight (1-u); u in [-1,0]: u = -v, weight (1-v) */
    ld u = gx[i], wt = gw[i] * (1.0L - u);
    for (int sg = -1; sg <= 1; sg += 2) {
      ld s = ((ld)d + sg * u) * h;
      ld e = expl(-rho * rho / (4.0L * alpha * s));
      ld is32 = 1.0L / (s * sqrtl(s));
      sV += wt * cG * is32 * e;
      sK += wt * cK * is32 / s * e;
    }
  }
  out[0] = h * h * sV;
  out[1] = h * h * sK;
}

static ld hat_integral(ld rho, int d, ld h, ld alpha, int which) {
  ld o[2];
  hat_integrals(rho, d, h, alpha, o);
  return o[which];
}

/* Temporal integral modes: 0 = closed form for d <= 16, hat quadrature above; 1 = closed form
 * for every d; 2 = hat quadrature for every d >= 2. */
static int use_hat(int d, int mode) {
  if (d < 2) return 0;
  if (mode == 1) return 0;
  if (mode == 2) return 1;
  return d > 16;
}

/* V^d(r) of Sec. 3.1 (d = 0: eq. for V^0; d >= 1: second difference of G^{dtau dt}). */
ld or_Vd(ld rho, int d, ld h, ld alpha, int mode) {
  if (use_hat(d, mode)) return hat_integral(rho, d, h, alpha, 0);
  if (d == 0) return h * or_g1(rho, 0.0L, alpha) - or_F(rho, h, alpha) + or_F(rho, 0.0L, alpha);
  return 2.0L * or_F(rho, d * h, alpha) - or_F(rho, (d + 1) * h, alpha) -
         or_F(rho, (d - 1) * h, alpha);
}

/* K^d(r) / (r . n_y) of Sec. 3.2. */
ld or_Kd_rn(ld rho, int d, ld h, ld alpha, int mode) {
  if (use_hat(d, mode)) return hat_integral(rho, d, h, alpha, 1);
  if (d == 0)
    return h * or_g1n_rn(rho, 0.0L, alpha) - or_Fn_rn(rho, h, alpha) + or_Fn_rn(rho, 0.0L, alpha);
  return 2.0L * or_Fn_rn(rho, d * h, alpha) - or_Fn_rn(rho, (d + 1) * h, alpha) -
         or_Fn_rn(rho, (d - 1) * h, alpha);
}

/* D^{2,d}(r) of Sec. 3.3 (second part of the hypersingular operator, eq. for D^{2,d}):
 *   d = 0:  alpha int_0^h G(r, t) dt = erfc(z_1) / (4 pi rho),
 *   d >= 1: alpha [int_{dh}^{(d+1)h} G(r, s) ds - int_{(d-1)h}^{dh} G(r, s) ds]
 *         = [erfc(z_{d+1}) - 2 erfc(z_d) + erfc(z_{d-1})] / (4 pi rho),   erfc(z_0) = 0,
 * with z_i = rho / (2 sqrt(alpha i h)): the second difference of -alpha G^{dt} = alpha G^{dtau},
 * using int_0^delta G(r, s) ds = erfc(z) / (4 pi alpha rho).  Where all arguments are below 1 the
 * same difference is taken of -erf (erf(z_0) = 1), since the erfc values then sit near 1. */
ld or_D2d(ld rho, int d, ld h, ld alpha) {
  const ld c = 1.0L / (4.0L * PI_L * rho);
  if (d == 0) return erfcl(rho / (2.0L * sqrtl(alpha * h))) * c;
  const ld zp = rho / (2.0L * sqrtl(alpha * (d + 1) * h)), z0 = rho / (2.0L * sqrtl(alpha * d * h));
  if (d >= 2) {
    const ld zm = rho / (2.0L * sqrtl(alpha * (d - 1) * h));
    if (zm < 1.0L) return -(erfl(zp) - 2.0L * erfl(z0) + erfl(zm)) * c;
    return (erfcl(zp) - 2.0L * erfcl(z0) + erfcl(zm)) * c;
  }
  return (erfcl(zp) - 2.0L * erfcl(z0)) * c;
}

/* ------------------------------------------------------------------------------------------ */
/* Spatial quadrature (Sec. 3.1 "Galerkin weights", Sec. 5.2).                                 */
/* Reference triangle T = {(x1, x2): 0 <= x2 <= x1 <= 1}, mapped by                             */
/*   chi(x) = v0 + x1 (v1 - v0) + x2 (v2 - v1),  |det| = 2 * area.                              */
/* ------------------------------------------------------------------------------------------ */

/* Radon's 7-point degree-5 rule in barycentric coordinates, weights summing to 1. */
static void radon7(ld lam[7][3], ld w[7]) {
  ld s15 = sqrtl(15.0L);
  ld a = (6.0L - s15) / 21.0L, b = (6.0L + s15) / 21.0L;
  ld wa = (155.0L - s15) / 1200.0L, wb = (155.0L + s15) / 1200.0L;
  ld L[7][3] = {{1.0L / 3, 1.0L / 3, 1.0L / 3},
                {a, a, 1 - 2 * a}, {a, 1 - 2 * a, a}, {1 - 2 * a, a, a},
                {b, b, 1 - 2 * b}, {b, 1 - 2 * b, b}, {1 - 2 * b, b, b}};
  ld W[7] = {9.0L / 40.0L, wa, wa, wa, wb, wb, wb};
  memcpy(lam, L, sizeof(L));
  memcpy(w, W, sizeof(W));
}

/* Triangle rules in barycentric coordinates, weights summing to 1.
 * kind 0: Radon 7 points (order ignored).  kind 1: collapsed (Duffy) Gauss product rule with
 * order x order points.  Returns the number of points written (caller supplies room). */
int or_triangle_rule(int kind, int order, double *lam_out, double *w_out) {
  if (kind == 0) {
    ld lam[7][3], w[7];
    radon7(lam, w);
    for (int i = 0; i < 7; ++i) {
      for (int k = 0; k < 3; ++k) lam_out[3 * i + k] = (double)lam[i][k];
      w_out[i] = (double)w[i];
    }
    return 7;
  }
  ld gx[64], gw[64];
  if (order < 1 || order > 64) return -1;
  gauss_legendre01(order, gx, gw);
  int c = 0;
  for (int i = 0; i < order; ++i)
    for (int j = 0; j < order; ++j) {
      ld x1 = gx[i], x2 = gx[i] * gx[j]; /* point of T, Jacobian x1 */
      lam_out[3 * c + 0] = (double)(1.0L - x1);
      lam_out[3 * c + 1] = (double)(x1 - x2);
      lam_out[3 * c + 2] = (double)x2;
      w_out[c] = (double)(2.0L * gw[i] * gw[j] * x1); /* |T| = 1/2 -> normalise to 1 */
      ++c;
    }
  return c;
}

/* Sauter-Schwab regularising maps [0,1]^4 -> T x T for the three touching configurations
 * (Sauter & Schwab, Boundary Element Methods, Sec. 5.2): identical panels (6 maps), a common
 * edge (5 maps; the shared edge is the image of [(0,0),(1,0)] in both panels) and a common
 * vertex (2 maps; the shared vertex is the image of (0,0)).  Returns the Jacobian of map s. */
static ld ss_map(int cls, int s, ld xi, ld e1, ld e2, ld e3, ld xh[2], ld yh[2]) {
  switch (cls) {
    case 3: /* identical */
      switch (s) {
        case 0: xh[0] = xi; xh[1] = xi * (1 - e1 + e1 * e2);
                yh[0] = xi * (1 - e1 * e2 * e3); yh[1] = xi * (1 - e1); break;
        case 1: xh[0] = xi * (1 - e1 * e2 * e3); xh[1] = xi * (1 - e1);
                yh[0] = xi; yh[1] = xi * (1 - e1 + e1 * e2); break;
        case 2: xh[0] = xi; xh[1] = xi * e1 * (1 - e2 + e2 * e3);
                yh[0] = xi * (1 - e1 * e2); yh[1] = xi * e1 * (1 - e2); break;
        case 3: xh[0] = xi * (1 - e1 * e2); xh[1] = xi * e1 * (1 - e2);
                yh[0] = xi; yh[1] = xi * e1 * (1 - e2 + e2 * e3); break;
        case 4: xh[0] = xi * (1 - e1 * e2 * e3); xh[1] = xi * e1 * (1 - e2 * e3);
                yh[0] = xi; yh[1] = xi * e1 * (1 - e2); break;
        default: xh[0] = xi; xh[1] = xi * e1 * (1 - e2);
                 yh[0] = xi * (1 - e1 * e2 * e3); yh[1] = xi * e1 * (1 - e2 * e3); break;
      }
      return xi * xi * xi * e1 * e1 * e2;
    case 2: /* common edge */
      switch (s) {
        case 0: xh[0] = xi; xh[1] = xi * e1 * e3;
                yh[0] = xi * (1 - e1 * e2); yh[1] = xi * e1 * (1 - e2);
                return xi * xi * xi * e1 * e1;
        case 1: xh[0] = xi; xh[1] = xi * e1;
                yh[0] = xi * (1 - e1 * e2 * e3); yh[1] = xi * e1 * e2 * (1 - e3); break;
        case 2: xh[0] = xi * (1 - e1 * e2); xh[1] = xi * e1 * (1 - e2);
                yh[0] = xi; yh[1] = xi * e1 * e2 * e3; break;
        case 3: xh[0] = xi * (1 - e1 * e2 * e3); xh[1] = xi * e1 * e2 * (1 - e3);
                yh[0] = xi; yh[1] = xi * e1; break;
        default: xh[0] = xi * (1 - e1 * e2 * e3); xh[1] = xi * e1 * (1 - e2 * e3);
                 yh[0] = xi; yh[1] = xi * e1 * e2; break;
      }
      return xi * xi * xi * e1 * e1 * e2;
    default: /* common vertex */
      if (s == 0) { xh[0] = xi; xh[1] = xi * e1; yh[0] = xi * e2; yh[1] = xi * e2 * e3; }
      else { xh[0] = xi * e2; xh[1] = xi * e2 * e3; yh[0] = xi; yh[1] = xi * e1; }
      return xi * xi * xi * e2;
  }
}

static int ss_nmaps(int cls) { return cls == 3 ? 6 : (cls == 2 ? 5 : 2); }

/* Regularised rule for class cls (3 identical, 2 edge, 1 vertex) with order^4 points per map.
 * Writes reference points (x1, x2) of both panels and weights w * J (summing to 1/4 = |T|^2).
 * Returns the number of points. */
int or_ss_rule(int cls, int order, double *xh_out, double *yh_out, double *w_out) {
  ld gx[64], gw[64];
  if (order < 1 || order > 64 || cls < 1 || cls > 3) return -1;
  gauss_legendre01(order, gx, gw);
  int c = 0;
  for (int s = 0; s < ss_nmaps(cls); ++s)
    for (int a = 0; a < order; ++a)
      for (int b = 0; b < order; ++b)
        for (int e = 0; e < order; ++e)
          for (int f = 0; f < order; ++f) {
            ld xh[2], yh[2];
            ld J = ss_map(cls, s, gx[f], gx[a], gx[b], gx[e], xh, yh);
            xh_out[2 * c] = (double)xh[0]; xh_out[2 * c + 1] = (double)xh[1];
            yh_out[2 * c] = (double)yh[0]; yh_out[2 * c + 1] = (double)yh[1];
            w_out[c] = (double)(gw[a] * gw[b] * gw[e] * gw[f] * J);
            ++c;
          }
  return c;
}

/* ---- mesh helpers ---- */
typedef struct {
  ld v[3][3]; /* vertex coordinates */
  ld area;
  ld n[3]; /* outward unit normal */
} tri_t;

static void make_tri(const double *verts, const int32_t *t, tri_t *T) {
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) T->v[k][c] = (ld)verts[3 * t[k] + c];
  ld e1[3], e2[3], cr[3];
  for (int c = 0; c < 3; ++c) { e1[c] = T->v[1][c] - T->v[0][c]; e2[c] = T->v[2][c] - T->v[0][c]; }
  cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
  cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
  cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
  ld nn = sqrtl(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  T->area = 0.5L * nn;
  for (int c = 0; c < 3; ++c) T->n[c] = cr[c] / nn;
}

/* Point of the panel whose vertices are v[p[0]], v[p[1]], v[p[2]] at reference point (x1, x2). */
static void ref_to_phys(const tri_t *T, const int p[3], ld x1, ld x2, ld out[3]) {
  for (int c = 0; c < 3; ++c)
    out[c] = T->v[p[0]][c] + x1 * (T->v[p[1]][c] - T->v[p[0]][c]) +
             x2 * (T->v[p[2]][c] - T->v[p[1]][c]);
}

/* Classify the ordered pair (test a, trial b) by shared vertex indices and find local vertex
 * orders pa, pb such that the shared vertices come first, in the same order, in both panels.
 * Returns the number of shared vertices (0 separated, 1 vertex, 2 edge, 3 identical). */
static int classify(const int32_t *ta, const int32_t *tb, int pa[3], int pb[3]) {
  int shared_a[3], shared_b[3], ns = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (ta[i] == tb[j]) { shared_a[ns] = i; shared_b[ns] = j; ++ns; }
  if (ns == 3) {
    for (int i = 0; i < 3; ++i) { pa[i] = i; pb[i] = i; }
    /* identical panel: same vertex order in both (tb == ta as sets; use ta's order) */
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (tb[j] == ta[i]) pb[i] = j;
    return 3;
  }
  if (ns == 0) {
    for (int i = 0; i < 3; ++i) { pa[i] = i; pb[i] = i; }
    return 0;
  }
  int used_a[3] = {0, 0, 0}, used_b[3] = {0, 0, 0};
  for (int k = 0; k < ns; ++k) {
    pa[k] = shared_a[k]; pb[k] = shared_b[k];
    used_a[shared_a[k]] = 1; used_b[shared_b[k]] = 1;
  }
  int ca = ns, cb = ns;
  for (int i = 0; i < 3; ++i) {
    if (!used_a[i]) pa[ca++] = i;
    if (!used_b[i]) pb[cb++] = i;
  }
  return ns;
}

/* Quadrature points of one ordered panel pair: physical x (test), y (trial), weight W (the
 * physical measure ds_x ds_y carried by the point), and the trial p1 basis values phi[k] for the
 * trial panel's ORIGINAL local vertex k.  Returns the count.  cap bounds the arrays. */
typedef struct {
  ld x[3], y[3], W, phi[3], phix[3]; /* phix: test p1 basis values, test panel's own vertex order */
} qpt_t;

static ld *g_ss_x[4], *g_ss_y[4], *g_ss_w[4];
static int g_ss_n[4] = {0, 0, 0, 0}, g_ss_order = -1;

/* Largest number of points one panel pair can carry at regularised order M. */
static int max_points(int ss_order) {
  int m4 = ss_order * ss_order * ss_order * ss_order;
  return 6 * m4 > 49 ? 6 * m4 : 49;
}
static ld g_r7[7][3], g_w7[7];

static void prepare_rules(int ss_order) {
  if (g_ss_order == ss_order) return;
  radon7(g_r7, g_w7);
  for (int cls = 1; cls <= 3; ++cls) {
    free(g_ss_x[cls]); free(g_ss_y[cls]); free(g_ss_w[cls]);
    size_t np = (size_t)max_points(ss_order);
    g_ss_x[cls] = (ld *)malloc(sizeof(ld) * 2 * np);
    g_ss_y[cls] = (ld *)malloc(sizeof(ld) * 2 * np);
    g_ss_w[cls] = (ld *)malloc(sizeof(ld) * np);
  }
  ld gx[64], gw[64];
  gauss_legendre01(ss_order, gx, gw);
  for (int cls = 1; cls <= 3; ++cls) {
    int c = 0;
    for (int s = 0; s < ss_nmaps(cls); ++s)
      for (int a = 0; a < ss_order; ++a)
        for (int b = 0; b < ss_order; ++b)
          for (int e = 0; e < ss_order; ++e)
            for (int f = 0; f < ss_order; ++f) {
              ld xh[2], yh[2];
              ld J = ss_map(cls, s, gx[f], gx[a], gx[b], gx[e], xh, yh);
              g_ss_x[cls][2 * c] = xh[0]; g_ss_x[cls][2 * c + 1] = xh[1];
              g_ss_y[cls][2 * c] = yh[0]; g_ss_y[cls][2 * c + 1] = yh[1];
              g_ss_w[cls][c] = gw[a] * gw[b] * gw[e] * gw[f] * J;
              ++c;
            }
    g_ss_n[cls] = c;
  }
  g_ss_order = ss_order;
}

static int pair_points(const double *verts, const int32_t *tris, int a, int b, qpt_t *q) {
  tri_t A, B;
  make_tri(verts, tris + 3 * a, &A);
  make_tri(verts, tris + 3 * b, &B);
  int pa[3], pb[3];
  int cls = classify(tris + 3 * a, tris + 3 * b, pa, pb);
  int n = 0;
  if (cls == 0) {
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j < 7; ++j) {
        for (int c = 0; c < 3; ++c) {
          q[n].x[c] = g_r7[i][0] * A.v[0][c] + g_r7[i][1] * A.v[1][c] + g_r7[i][2] * A.v[2][c];
          q[n].y[c] = g_r7[j][0] * B.v[0][c] + g_r7[j][1] * B.v[1][c] + g_r7[j][2] * B.v[2][c];
        }
        q[n].W = g_w7[i] * g_w7[j] * A.area * B.area;
        for (int k = 0; k < 3; ++k) q[n].phi[k] = g_r7[j][k];
        for (int k = 0; k < 3; ++k) q[n].phix[k] = g_r7[i][k];
        ++n;
      }
    return n;
  }
  for (int i = 0; i < g_ss_n[cls]; ++i) {
    ld xh1 = g_ss_x[cls][2 * i], xh2 = g_ss_x[cls][2 * i + 1];
    ld yh1 = g_ss_y[cls][2 * i], yh2 = g_ss_y[cls][2 * i + 1];
    ref_to_phys(&A, pa, xh1, xh2, q[n].x);
    ref_to_phys(&B, pb, yh1, yh2, q[n].y);
    q[n].W = 4.0L * A.area * B.area * g_ss_w[cls][i];
    /* barycentric coordinates of the trial point w.r.t. the permuted vertices pb[0..2] */
    ld lam[3] = {1.0L - yh1, yh1 - yh2, yh2};
    for (int k = 0; k < 3; ++k) q[n].phi[pb[k]] = lam[k];
    ld lax[3] = {1.0L - xh1, xh1 - xh2, xh2};
    for (int k = 0; k < 3; ++k) q[n].phix[pa[k]] = lax[k];
    ++n;
  }
  return n;
}

/* Exposed for tests: the quadrature points of pair (a, b); returns count and class. */
int or_pair_points(const double *verts, const int32_t *tris, int a, int b, int ss_order,
                   double *x, double *y, double *W, double *phi, int *cls_out) {
  prepare_rules(ss_order);
  qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * max_points(ss_order));
  int pa[3], pb[3];
  *cls_out = classify(tris + 3 * a, tris + 3 * b, pa, pb);
  int n = pair_points(verts, tris, a, b, q);
  for (int i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) { x[3 * i + c] = (double)q[i].x[c]; y[3 * i + c] = (double)q[i].y[c]; }
    W[i] = (double)q[i].W;
    for (int k = 0; k < 3; ++k) phi[3 * i + k] = (double)q[i].phi[k];
  }
  free(q);
  return n;
}

/* ------------------------------------------------------------------------------------------ */
/* Assembly of V_h^d and K_h^d for the test rows `rows` (all trial panels, all d).             */
/*   V out: [n_t][n_rows][n_tris], K out: [n_t][n_rows][n_verts], both zero-initialised here.    */
/* method 0 ("direct"): per point pair, the exact temporal integral V^d(r), K^d(r) of each block */
/*   is evaluated (temporal mode tmode) and summed with the spatial weights.                    */
/* method 1 ("levels"): the paper's order -- loop over i_t = delta/h, evaluate G^{dtau dt} and   */
/*   its normal derivative once per point pair, scatter with the stencil of Tables 5.1/5.2.     */
/* ------------------------------------------------------------------------------------------ */
static void assemble_row_direct(const double *verts, const int32_t *tris, int nv, int ne, int row,
                                int rloc, int nrows, ld alpha, ld h, int nt, int tmode,
                                double *V, double *K, qpt_t *q, ld *vd, ld *kd, ld *fl) {
  tri_t B;
  /* levels needed by the closed form: 0 .. min(nt, 17) */
  int nlev = nt < 17 ? nt : 17;
  for (int m = 0; m < ne; ++m) {
    make_tri(verts, tris + 3 * m, &B);
    int n = pair_points(verts, tris, row, m, q);
    for (int d = 0; d < nt; ++d) { vd[d] = 0.0L; kd[3 * d] = kd[3 * d + 1] = kd[3 * d + 2] = 0.0L; }
    for (int i = 0; i < n; ++i) {
      ld r[3] = {q[i].x[0] - q[i].y[0], q[i].x[1] - q[i].y[1], q[i].x[2] - q[i].y[2]};
      ld rho = sqrtl(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      ld rn = r[0] * B.n[0] + r[1] * B.n[1] + r[2] * B.n[2];
      /* G^{dtau dt}(rho, l h) and its normal derivative / (r.n) at levels l = 0..nlev */
      for (int l = 0; l <= nlev; ++l) {
        fl[2 * l] = or_F(rho, l * h, alpha);
        fl[2 * l + 1] = or_Fn_rn(rho, l * h, alpha);
      }
      for (int d = 0; d < nt; ++d) {
        ld v, kr;
        if (use_hat(d, tmode)) {
          ld o[2];
          hat_integrals(rho, d, h, alpha, o);
          v = o[0];
          kr = o[1];
        } else if (d == 0) { /* eq. for V^0 and K^0 */
          v = h * or_g1(rho, 0.0L, alpha) - fl[2] + fl[0];
          kr = h * or_g1n_rn(rho, 0.0L, alpha) - fl[3] + fl[1];
        } else if (d + 1 <= nlev) { /* second differences of eq. for V^d and K^d */
          v = 2.0L * fl[2 * d] - fl[2 * (d + 1)] - fl[2 * (d - 1)];
          kr = 2.0L * fl[2 * d + 1] - fl[2 * (d + 1) + 1] - fl[2 * (d - 1) + 1];
        } else {
          v = or_Vd(rho, d, h, alpha, tmode);
          kr = or_Kd_rn(rho, d, h, alpha, tmode);
        }
        vd[d] += q[i].W * v;
        ld kv = q[i].W * rn * kr;
        for (int k = 0; k < 3; ++k) kd[3 * d + k] += kv * q[i].phi[k];
      }
    }
    for (int d = 0; d < nt; ++d) {
      V[((size_t)d * nrows + rloc) * ne + m] = (double)vd[d];
      for (int k = 0; k < 3; ++k)
        K[((size_t)d * nrows + rloc) * nv + tris[3 * m + k]] += (double)kd[3 * d + k];
    }
  }
}

/* One ordered panel pair (test a, trial b), every block: V_h^d[a][b] and the contributions of
 * panel b to row a of K_h^d through its local vertices k (out V[nt], K[nt][3]); the same
 * per-point temporal integrals as the direct assembly (temporal mode 0). */
int or_pair_blocks(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                   double T, int nt, int ss_order, int a, int b, double *V, double *K) {
  if (nt < 1 || a < 0 || b < 0 || a >= ne || b >= ne || nv < 3) return -1;
  prepare_rules(ss_order);
  qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * max_points(ss_order));
  tri_t B;
  make_tri(verts, tris + 3 * b, &B);
  const ld h = (ld)T / nt, al = (ld)alpha;
  int n = pair_points(verts, tris, a, b, q);
  for (int d = 0; d < nt; ++d) {
    ld vd = 0.0L, kd[3] = {0.0L, 0.0L, 0.0L};
    for (int i = 0; i < n; ++i) {
      ld r[3] = {q[i].x[0] - q[i].y[0], q[i].x[1] - q[i].y[1], q[i].x[2] - q[i].y[2]};
      ld rho = sqrtl(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      ld rn = r[0] * B.n[0] + r[1] * B.n[1] + r[2] * B.n[2];
      vd += q[i].W * or_Vd(rho, d, h, al, 0);
      ld kv = q[i].W * rn * or_Kd_rn(rho, d, h, al, 0);
      for (int k = 0; k < 3; ++k) kd[k] += kv * q[i].phi[k];
    }
    V[d] = (double)vd;
    for (int k = 0; k < 3; ++k) K[3 * d + k] = (double)kd[k];
  }
  free(q);
  return 0;
}

int or_assemble(const double *verts, int nv, const int32_t *tris, int ne, double alpha, double T,
                int nt, int ss_order, const int32_t *rows, int nrows, int method, int tmode,
                double *V, double *K) {
  if (nt < 1 || ne < 1 || nv < 3 || alpha <= 0 || T <= 0) return -1;
  prepare_rules(ss_order);
  memset(V, 0, sizeof(double) * (size_t)nt * nrows * ne);
  memset(K, 0, sizeof(double) * (size_t)nt * nrows * nv);
  ld h = (ld)T / (ld)nt, al = (ld)alpha;
  if (method == 0) {
#pragma omp parallel
    {
      qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * max_points(ss_order));
      ld *vd = (ld *)malloc(sizeof(ld) * nt);
      ld *kd = (ld *)malloc(sizeof(ld) * 3 * nt);
      ld *fl = (ld *)malloc(sizeof(ld) * 2 * (nt + 2));
#pragma omp for schedule(dynamic)
      for (int r = 0; r < nrows; ++r)
        assemble_row_direct(verts, tris, nv, ne, rows[r], r, nrows, al, h, nt, tmode, V, K, q, vd,
                            kd, fl);
      free(q); free(vd); free(kd); free(fl);
    }
    return 0;
  }
  /* levels: accumulate in long double per row, then round */
  ld *VL = (ld *)calloc((size_t)nt * nrows * ne, sizeof(ld));
  ld *KL = (ld *)calloc((size_t)nt * nrows * nv, sizeof(ld));
  for (int it = 0; it <= nt; ++it) {
    ld delta = it * h;
#pragma omp parallel
    {
      qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * max_points(ss_order));
      tri_t B;
#pragma omp for schedule(dynamic)
      for (int r = 0; r < nrows; ++r) {
        for (int m = 0; m < ne; ++m) {
          make_tri(verts, tris + 3 * m, &B);
          int n = pair_points(verts, tris, rows[r], m, q);
          ld val = 0.0L, vs = 0.0L, kval[3] = {0, 0, 0}, ks[3] = {0, 0, 0};
          for (int i = 0; i < n; ++i) {
            ld rr[3] = {q[i].x[0] - q[i].y[0], q[i].x[1] - q[i].y[1], q[i].x[2] - q[i].y[2]};
            ld rho = sqrtl(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]);
            ld rn = rr[0] * B.n[0] + rr[1] * B.n[1] + rr[2] * B.n[2];
            val += q[i].W * or_F(rho, delta, al);
            ld kv = q[i].W * rn * or_Fn_rn(rho, delta, al);
            for (int k = 0; k < 3; ++k) kval[k] += kv * q[i].phi[k];
            if (it == 0) {
              vs += q[i].W * h * or_g1(rho, 0.0L, al);
              ld ksv = q[i].W * rn * h * or_g1n_rn(rho, 0.0L, al);
              for (int k = 0; k < 3; ++k) ks[k] += ksv * q[i].phi[k];
            }
          }
          /* stencil of Tables 5.1 / 5.2 */
          for (int tgt = 0; tgt < 3; ++tgt) {
            int d;
            ld coef;
            if (tgt == 0) { if (it == 0) { d = 0; coef = 1.0L; } else { d = it - 1; coef = -1.0L; } }
            else if (tgt == 1) { if (it == 0 || it >= nt) continue; d = it; coef = 2.0L; }
            else { if (it >= nt - 1) continue; d = it + 1; coef = -1.0L; }
            VL[((size_t)d * nrows + r) * ne + m] += coef * val;
            for (int k = 0; k < 3; ++k)
              KL[((size_t)d * nrows + r) * nv + tris[3 * m + k]] += coef * kval[k];
          }
          if (it == 0) {
            VL[((size_t)0 * nrows + r) * ne + m] += vs;
            for (int k = 0; k < 3; ++k) KL[((size_t)0 * nrows + r) * nv + tris[3 * m + k]] += ks[k];
          }
        }
      }
      free(q);
    }
  }
  for (size_t i = 0; i < (size_t)nt * nrows * ne; ++i) V[i] = (double)VL[i];
  for (size_t i = 0; i < (size_t)nt * nrows * nv; ++i) K[i] = (double)KL[i];
  free(VL); free(KL);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Non-uniform time steps (the paper's closing outlook, Sec. 7; the block integrals of Sec. 3.1  */
/* and 3.2 at general interval endpoints).  Nodes 0 = t_0 < t_1 < ... < t_nt; test interval k is */
/* (t_k, t_{k+1}), trial interval i is (t_i, t_{i+1}), i <= k.  The block integral               */
/*   V^{k,i}(r) = int_{I_k} int_{I_i} G_alpha(rho, t - tau) dtau dt                             */
/* is, since d^2 G^{dtau dt} / d delta^2 = -G_alpha, for i < k the four-term difference           */
/*   F(t_k - t_i) + F(t_{k+1} - t_{i+1}) - F(t_{k+1} - t_i) - F(t_k - t_{i+1})   (F = G^{dtau dt}),  */
/* and for i = k (tau < t only): h_k G^{dtau}(rho, 0) - F(h_k) + F(0); K^{k,i} / (r . n_y) the same  */
/* with the normal derivatives.  Where the four terms cancel (the gap s1 = t_k - t_{i+1} at least */
/* the width s4 - s1 of the support, s4 = t_{k+1} - t_i), the same integral is evaluated as      */
/*   int_{s1}^{s4} w(s) G_alpha(rho, s) ds,                                                      */
/* w the trapezoid that is the convolution of the two interval indicators (rising on            */
/* [s1, s1 + min(h_k, h_i)], flat at min(h_k, h_i), falling to 0 at s4), by Gauss-Legendre with   */
/* NU_NT nodes on each of its three linear pieces (the integrand is analytic there: its only     */
/* singularity, s = 0, lies at least one support width to the left).                           */
/* ------------------------------------------------------------------------------------------ */
#define NU_NT 16
static void nu_trapezoid(ld rho, ld s1, ld a, ld b, ld alpha, ld out[2]) {
  static ld gx[NU_NT], gw[NU_NT];
  static int ready = 0;
  if (!ready) {
#pragma omp critical(oracle_nu_init)
    {
      if (!ready) {
        gauss_legendre01(NU_NT, gx, gw);
        __sync_synchronize();
        ready = 1;
      }
    }
  }
  const ld cG = 1.0L / ((4.0L * PI_L * alpha) * sqrtl(4.0L * PI_L * alpha));
  const ld cK = 1.0L / (16.0L * PI_L * alpha * sqrtl(PI_L * alpha));
  const ld mn = a < b ? a : b, mx = a < b ? b : a;
  /* pieces [s1, s1 + mn] (w = s - s1), [s1 + mn, s1 + mx] (w = mn), [s1 + mx, s1 + a + b] (w = s4 - s) */
  const ld lo[3] = {s1, s1 + mn, s1 + mx}, len[3] = {mn, mx - mn, mn};
  ld sV = 0.0L, sK = 0.0L;
  for (int piece = 0; piece < 3; ++piece) {
    if (len[piece] <= 0.0L) continue;
    for (int j = 0; j < NU_NT; ++j) {
      const ld s = lo[piece] + len[piece] * gx[j];
      const ld wt = piece == 0 ? s - s1 : (piece == 1 ? mn : s1 + a + b - s);
      const ld e = expl(-rho * rho / (4.0L * alpha * s));
      const ld is32 = 1.0L / (s * sqrtl(s));
      sV += len[piece] * gw[j] * wt * cG * is32 * e;
      sK += len[piece] * gw[j] * wt * cK * is32 / s * e;
    }
  }
  out[0] = sV;
  out[1] = sK;
}

/* V^{k,i}(r) (out[0]) and K^{k,i}(r) / (r . n_y) (out[1]) on the grid t (nt + 1 nodes). */
void or_nu_block(ld rho, int k, int i, const double *t, ld alpha, ld out[2]) {
  const ld hk = (ld)t[k + 1] - (ld)t[k], hi = (ld)t[i + 1] - (ld)t[i];
  if (i == k) {
    out[0] = hk * or_g1(rho, 0.0L, alpha) - or_F(rho, hk, alpha) + or_F(rho, 0.0L, alpha);
    out[1] = hk * or_g1n_rn(rho, 0.0L, alpha) - or_Fn_rn(rho, hk, alpha) + or_Fn_rn(rho, 0.0L, alpha);
    return;
  }
  const ld s1 = (ld)t[k] - (ld)t[i + 1], s4 = (ld)t[k + 1] - (ld)t[i];
  if (s1 >= s4 - s1) {
    nu_trapezoid(rho, s1, hk, hi, alpha, out);
    return;
  }
  const ld d1 = (ld)t[k] - (ld)t[i], d2 = (ld)t[k + 1] - (ld)t[i + 1];
  out[0] = or_F(rho, d1, alpha) + or_F(rho, d2, alpha) - or_F(rho, s4, alpha) - or_F(rho, s1, alpha);
  out[1] = or_Fn_rn(rho, d1, alpha) + or_Fn_rn(rho, d2, alpha) - or_Fn_rn(rho, s4, alpha) -
           or_Fn_rn(rho, s1, alpha);
}

/* Blocks V^{k,i}_h (p0 x p0) and K^{k,i}_h (p0 x p1) of the test rows `rows` on the grid t, all
 * 0 <= i <= k < nt, packed by block rows: block (k, i) at index k (k + 1) / 2 + i.
 * V out: [nb][nrows][ne], K out: [nb][nrows][nv], nb = nt (nt + 1) / 2.  The same spatial rules
 * as or_assemble. */
int or_assemble_nonuniform(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                           const double *t, int nt, int ss_order, const int32_t *rows, int nrows,
                           double *V, double *K) {
  if (nt < 1 || ne < 1 || nv < 3 || alpha <= 0 || t[0] != 0.0) return -1;
  for (int k = 0; k < nt; ++k)
    if (!(t[k + 1] > t[k])) return -1;
  prepare_rules(ss_order);
  const int nb = nt * (nt + 1) / 2;
  memset(V, 0, sizeof(double) * (size_t)nb * nrows * ne);
  memset(K, 0, sizeof(double) * (size_t)nb * nrows * nv);
  const ld al = (ld)alpha;
#pragma omp parallel
  {
    qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * max_points(ss_order));
    ld *vd = (ld *)malloc(sizeof(ld) * nb);
    ld *kd = (ld *)malloc(sizeof(ld) * 3 * nb);
    tri_t B;
#pragma omp for schedule(dynamic)
    for (int r = 0; r < nrows; ++r) {
      for (int m = 0; m < ne; ++m) {
        make_tri(verts, tris + 3 * m, &B);
        const int n = pair_points(verts, tris, rows[r], m, q);
        for (int e = 0; e < nb; ++e) { vd[e] = 0.0L; kd[3 * e] = kd[3 * e + 1] = kd[3 * e + 2] = 0.0L; }
        for (int j = 0; j < n; ++j) {
          const ld rr[3] = {q[j].x[0] - q[j].y[0], q[j].x[1] - q[j].y[1], q[j].x[2] - q[j].y[2]};
          const ld rho = sqrtl(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2]);
          const ld rn = rr[0] * B.n[0] + rr[1] * B.n[1] + rr[2] * B.n[2];
          for (int k = 0; k < nt; ++k)
            for (int i = 0; i <= k; ++i) {
              ld o[2];
              or_nu_block(rho, k, i, t, al, o);
              const int e = k * (k + 1) / 2 + i;
              vd[e] += q[j].W * o[0];
              const ld kv = q[j].W * rn * o[1];
              for (int c = 0; c < 3; ++c) kd[3 * e + c] += kv * q[j].phi[c];
            }
        }
        for (int e = 0; e < nb; ++e) {
          V[((size_t)e * nrows + r) * ne + m] = (double)vd[e];
          for (int c = 0; c < 3; ++c)
            K[((size_t)e * nrows + r) * nv + tris[3 * m + c]] += (double)kd[3 * e + c];
        }
      }
    }
    free(q); free(vd); free(kd);
  }
  return 0;
}

/* Per-point block functions on a grid (tests): out[e] = V^{k,i}(rho_e) (which 0) or
 * K^{k,i}(rho_e) / (r . n_y) (which 1) for the blocks (k_e, i_e). */
void or_nu_blockfun(int which, const double *rho, const int32_t *k, const int32_t *i, int n,
                    const double *t, double alpha, double *out) {
  for (int e = 0; e < n; ++e) {
    ld o[2];
    or_nu_block((ld)rho[e], k[e], i[e], t, (ld)alpha, o);
    out[e] = (double)o[which];
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Plain double-precision assembly in the paper's order (Sec. 5.1, the listing of the assembly  */
/* structure; Tables 5.1/5.2): for each level i_t = 0 .. n_t, the test rows (OpenMP, dynamic),  */
/* for each trial panel the kernel G^{dtau dt}(r, i_t h) and its normal derivative at every      */
/* quadrature point in double, summed with the weights and added to blocks i_t - 1, i_t,         */
/* i_t + 1 with the multipliers -1, 2, -1 (block 0 at level 0 with 1, plus the h G^{dtau}(r, 0)  */
/* terms of V^0 and K^0).  No long double and no hat quadrature: this is the method as the paper */
/* runs it, the CPU baseline that is timed, not the parity reference (its second differences    */
/* lose digits as d grows).  The small-z series of the double-layer bracket is kept, since the   */
/* closed form is 0/0 there.  nthreads > 0 fixes the OpenMP team size.                          */
/* ------------------------------------------------------------------------------------------ */
static const double PI_D = 3.14159265358979323846;

static int shares_vertex(const int32_t *ta, const int32_t *tb) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (ta[i] == tb[j]) return 1;
  return 0;
}

/* G^{dtau dt}(rho, delta) (out[0]) and alpha dG^{dtau dt}/dn_y / (r . n_y) (out[1]) in double,
 * sharing one erf and one exp (formula summary, Sec. 4); limits at delta = 0 */
static void f64_F_Fn(double rho, double delta, double alpha, double out[2]) {
  if (delta <= 0.0) {
    out[0] = rho / (8.0 * PI_D * alpha * alpha);
    out[1] = -1.0 / (8.0 * PI_D * alpha * rho);
    return;
  }
  const double z = rho / (2.0 * sqrt(alpha * delta));
  const double ez = erf(z), gz = exp(-z * z);
  out[0] = ((rho / (2.0 * alpha * alpha) + delta / (alpha * rho)) * ez +
            sqrt(delta / (PI_D * alpha * alpha * alpha)) * gz) / (4.0 * PI_D);
  if (z < 0.5) { /* the series of B(z), the closed form being 0/0 there */
    double z2 = z * z, term = z, sum = 0.0;
    for (int n = 0; n < 14; ++n) {
      sum += term / ((double)(2 * n + 1) * (double)(2 * n + 3));
      term *= -z2 / (double)(n + 1);
    }
    out[1] = -(4.0 / sqrt(PI_D)) * sum / (8.0 * PI_D * alpha * rho);
  } else {
    out[1] = -((1.0 / (2.0 * alpha) - delta / (rho * rho)) * ez +
               sqrt(delta) / (rho * sqrt(PI_D * alpha)) * gz) / (4.0 * PI_D * rho);
  }
}

int or_assemble_plain(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                      double T, int nt, int ss_order, const int32_t *rows, int nrows, int nthreads,
                      double *V, double *K) {
  if (nt < 1 || ne < 1 || nv < 3 || alpha <= 0 || T <= 0) return -1;
  prepare_rules(ss_order);
  memset(V, 0, sizeof(double) * (size_t)nt * nrows * ne);
  memset(K, 0, sizeof(double) * (size_t)nt * nrows * nv);
  const double h = T / nt;
  const int np = max_points(ss_order);
  double r7[7][3], w7[7];
  for (int i = 0; i < 7; ++i) {
    w7[i] = (double)g_w7[i];
    for (int k = 0; k < 3; ++k) r7[i][k] = (double)g_r7[i][k];
  }
  double *area = (double *)malloc(sizeof(double) * ne);
  for (int m = 0; m < ne; ++m) {
    tri_t A;
    make_tri(verts, tris + 3 * m, &A);
    area[m] = (double)A.area;
  }
  /* the quadrature points of every pair are formed per level, as the listing does per pair */
  for (int it = 0; it <= nt; ++it) {
    const double delta = it * h;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    {
      qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * np);
      double *x = (double *)malloc(sizeof(double) * 11 * np);
      tri_t B;
#pragma omp for schedule(dynamic)
      for (int r = 0; r < nrows; ++r) {
        for (int m = 0; m < ne; ++m) {
          make_tri(verts, tris + 3 * m, &B);
          const double nb[3] = {(double)B.n[0], (double)B.n[1], (double)B.n[2]};
          int n;
          if (!shares_vertex(tris + 3 * rows[r], tris + 3 * m)) {
            /* separated pair: the 7-point rule on both panels, mapped in double (Sec. 5.2) */
            n = 49;
            for (int i = 0; i < 7; ++i)
              for (int j = 0; j < 7; ++j) {
                const int e = 7 * i + j;
                for (int c = 0; c < 3; ++c) {
                  double xc = 0.0, yc = 0.0;
                  for (int k = 0; k < 3; ++k) {
                    xc += r7[i][k] * verts[3 * tris[3 * rows[r] + k] + c];
                    yc += r7[j][k] * verts[3 * tris[3 * m + k] + c];
                  }
                  x[c * np + e] = xc - yc;
                }
                x[3 * np + e] = w7[i] * w7[j] * area[rows[r]] * area[m];
                for (int k = 0; k < 3; ++k) x[(4 + k) * np + e] = r7[j][k];
              }
          } else {
            n = pair_points(verts, tris, rows[r], m, q);
            for (int i = 0; i < n; ++i) { /* structure of arrays in double */
              for (int c = 0; c < 3; ++c) x[c * np + i] = (double)(q[i].x[c] - q[i].y[c]);
              x[3 * np + i] = (double)q[i].W;
              for (int k = 0; k < 3; ++k) x[(4 + k) * np + i] = (double)q[i].phi[k];
            }
          }
          double val = 0.0, vs = 0.0, kval[3] = {0, 0, 0}, ks[3] = {0, 0, 0};
          for (int i = 0; i < n; ++i) {
            const double r0 = x[i], r1 = x[np + i], r2 = x[2 * np + i], W = x[3 * np + i];
            const double rho = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
            const double rn = r0 * nb[0] + r1 * nb[1] + r2 * nb[2];
            double f[2];
            f64_F_Fn(rho, delta, alpha, f);
            val += W * f[0];
            const double kv = W * rn * f[1];
            for (int k = 0; k < 3; ++k) kval[k] += kv * x[(4 + k) * np + i];
            if (it == 0) {
              vs += W * h / (4.0 * PI_D * alpha * rho);
              const double ksv = W * rn * h / (4.0 * PI_D * rho * rho * rho);
              for (int k = 0; k < 3; ++k) ks[k] += ksv * x[(4 + k) * np + i];
            }
          }
          /* multipliers of Tables 5.1 / 5.2 */
          for (int tgt = 0; tgt < 3; ++tgt) {
            int d;
            double coef;
            if (tgt == 0) { if (it == 0) { d = 0; coef = 1.0; } else { d = it - 1; coef = -1.0; } }
            else if (tgt == 1) { if (it == 0 || it >= nt) continue; d = it; coef = 2.0; }
            else { if (it >= nt - 1) continue; d = it + 1; coef = -1.0; }
            V[((size_t)d * nrows + r) * ne + m] += coef * val;
            for (int k = 0; k < 3; ++k)
              K[((size_t)d * nrows + r) * nv + tris[3 * m + k]] += coef * kval[k];
          }
          if (it == 0) {
            V[(size_t)r * ne + m] += vs;
            for (int k = 0; k < 3; ++k) K[(size_t)r * nv + tris[3 * m + k]] += ks[k];
          }
        }
      }
      free(q);
      free(x);
    }
  }
  free(area);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Galerkin blocks of the second part of the hypersingular operator (Sec. 3.3):                */
/*   D2^d[i][j] = int int n(x) . n(y) phi^1_i(x) phi^1_j(y) D^{2,d}(x - y) ds_y ds_x,           */
/* every ordered panel pair with the same rules as V and K.  D2 out: [n_t][n_verts][n_verts].    */
/* ------------------------------------------------------------------------------------------ */
/* which = 0: V^{11} blocks, the single layer between p1 test and p1 trial functions (the matrix
 * of the paper's operator preconditioner for D_h, Sec. 6.1): kernel V^d(r), no normal factor;
 * which = 1: D^2 blocks as above. */
static int assemble_p1p1(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                         double T, int nt, int ss_order, int which, double *D2);

int or_assemble_d2(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                   double T, int nt, int ss_order, double *D2) {
  return assemble_p1p1(verts, nv, tris, ne, alpha, T, nt, ss_order, 1, D2);
}

int or_assemble_v11(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                    double T, int nt, int ss_order, double *V11) {
  return assemble_p1p1(verts, nv, tris, ne, alpha, T, nt, ss_order, 0, V11);
}

static int assemble_p1p1(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                         double T, int nt, int ss_order, int which, double *D2) {
  if (nt < 1 || ne < 1 || nv < 3 || alpha <= 0 || T <= 0) return -1;
  prepare_rules(ss_order);
  ld h = (ld)T / (ld)nt, al = (ld)alpha;
  ld *DL = (ld *)calloc((size_t)nt * nv * nv, sizeof(ld));
#pragma omp parallel
  {
    qpt_t *q = (qpt_t *)malloc(sizeof(qpt_t) * max_points(ss_order));
    ld *acc = (ld *)malloc(sizeof(ld) * 9 * nt);
    ld *rows = (ld *)malloc(sizeof(ld) * 3 * nt * (size_t)nv); /* the test panel's three rows */
    tri_t A, B;
#pragma omp for schedule(dynamic)
    for (int a = 0; a < ne; ++a) {
      make_tri(verts, tris + 3 * a, &A);
      for (size_t i = 0; i < 3 * (size_t)nt * nv; ++i) rows[i] = 0.0L;
      for (int b = 0; b < ne; ++b) {
        make_tri(verts, tris + 3 * b, &B);
        const ld nn = which ? A.n[0] * B.n[0] + A.n[1] * B.n[1] + A.n[2] * B.n[2] : 1.0L;
        int n = pair_points(verts, tris, a, b, q);
        for (int i = 0; i < 9 * nt; ++i) acc[i] = 0.0L;
        for (int i = 0; i < n; ++i) {
          ld r[3] = {q[i].x[0] - q[i].y[0], q[i].x[1] - q[i].y[1], q[i].x[2] - q[i].y[2]};
          ld rho = sqrtl(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
          for (int d = 0; d < nt; ++d) {
            ld v = q[i].W * (which ? or_D2d(rho, d, h, al) : or_Vd(rho, d, h, al, 0));
            for (int k = 0; k < 3; ++k)
              for (int l = 0; l < 3; ++l) acc[9 * d + 3 * k + l] += v * q[i].phix[k] * q[i].phi[l];
          }
        }
        for (int d = 0; d < nt; ++d)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
              rows[((size_t)k * nt + d) * nv + tris[3 * b + l]] += nn * acc[9 * d + 3 * k + l];
      }
#pragma omp critical(oracle_d2_rows)
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < nt; ++d)
          for (int j = 0; j < nv; ++j)
            DL[((size_t)d * nv + tris[3 * a + k]) * nv + j] += rows[((size_t)k * nt + d) * nv + j];
    }
    free(q); free(acc); free(rows);
  }
  for (size_t i = 0; i < (size_t)nt * nv * nv; ++i) D2[i] = (double)DL[i];
  free(DL);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Representation formula (Sec. 3.5): u(x, t) = (V~ w)(x, t) - (W u)(x, t) at points off Gamma. */
/* w: [n_t][n_tris] (p0 x p0 coefficients), u: [n_t][n_verts] (p1 x p0 coefficients),           */
/* pts: [P][4] = (x, y, z, t) with 0 <= t <= T.  The spatial rule is the same triangle rule as    */
/* for separated pairs (kind/order as or_triangle_rule).  Outputs sl[P], dl[P].                   */
/* ------------------------------------------------------------------------------------------ */
/* int_{tau1}^{tau2} G(rho, t - tau) dtau = g1(rho, t - tau2) - g1(rho, t - tau1), in the erfc form. */
static ld time_int_G(ld rho, ld s_lo, ld s_hi, ld alpha) {
  /* = [erf(z_lo) - erf(z_hi)]/(4 pi alpha rho) = [erfc(z_hi) - erfc(z_lo)]/(4 pi alpha rho) */
  ld zl = s_lo > 0 ? rho / (2.0L * sqrtl(alpha * s_lo)) : INFINITY;
  ld zh = rho / (2.0L * sqrtl(alpha * s_hi));
  ld el = s_lo > 0 ? erfcl(zl) : 0.0L;
  return (erfcl(zh) - el) / (4.0L * PI_L * alpha * rho);
}

static ld time_int_Gn_rn(ld rho, ld s_lo, ld s_hi, ld alpha) {
  return or_g1n_rn(rho, s_lo, alpha) - or_g1n_rn(rho, s_hi, alpha);
}

int or_repr(const double *verts, int nv, const int32_t *tris, int ne, double alpha, double T,
            int nt, const double *w, const double *u, const double *pts, int P, int rule_kind,
            int rule_order, double *sl, double *dl) {
  (void)nv;
  double lam[3 * 4096], wq[4096];
  int nq = or_triangle_rule(rule_kind, rule_order, lam, wq);
  if (nq <= 0) return -1;
  ld h = (ld)T / nt, al = (ld)alpha;
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < P; ++p) {
    ld x[3] = {pts[4 * p], pts[4 * p + 1], pts[4 * p + 2]}, t = pts[4 * p + 3];
    int k = (int)floorl(t / h);
    if (k > nt) k = nt;
    ld eps = t - k * h;
    if (eps < 0) eps = 0;
    ld accs = 0.0L, accd = 0.0L;
    for (int j = 0; j < ne; ++j) {
      tri_t B;
      make_tri(verts, tris + 3 * j, &B);
      for (int q = 0; q < nq; ++q) {
        ld y[3], r[3];
        for (int c = 0; c < 3; ++c) {
          y[c] = lam[3 * q] * B.v[0][c] + lam[3 * q + 1] * B.v[1][c] + lam[3 * q + 2] * B.v[2][c];
          r[c] = x[c] - y[c];
        }
        ld rho = sqrtl(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        ld rn = r[0] * B.n[0] + r[1] * B.n[1] + r[2] * B.n[2];
        ld Wq = wq[q] * B.area;
        ld ws = 0.0L, wd[3] = {0, 0, 0};
        /* past intervals i = 1..k (0-based index i-1), s ranges (t - t_i, t - t_{i-1}) */
        for (int i = 1; i <= k && i <= nt; ++i) {
          ld s_lo = t - i * h, s_hi = t - (i - 1) * h;
          ws += w[(size_t)(i - 1) * ne + j] * time_int_G(rho, s_lo, s_hi, al);
          ld gn = time_int_Gn_rn(rho, s_lo, s_hi, al);
          for (int c = 0; c < 3; ++c) wd[c] += u[(size_t)(i - 1) * nv + tris[3 * j + c]] * gn;
        }
        /* current interval k+1 (0-based k), s in (0, eps) */
        if (eps > 0 && k < nt) {
          ws += w[(size_t)k * ne + j] * time_int_G(rho, 0.0L, eps, al);
          ld gn = time_int_Gn_rn(rho, 0.0L, eps, al);
          for (int c = 0; c < 3; ++c) wd[c] += u[(size_t)k * nv + tris[3 * j + c]] * gn;
        }
        accs += Wq * ws;
        accd += Wq * rn * (lam[3 * q] * wd[0] + lam[3 * q + 1] * wd[1] + lam[3 * q + 2] * wd[2]);
      }
    }
    sl[p] = (double)accs;
    dl[p] = (double)accd;
  }
  return 0;
}

/* The same on a non-uniform time grid t[0] = 0 < t[1] < ... < t[nt] (the paper's outlook, Sec. 7,
 * with the time integrals of Sec. 3.5 over general intervals): w, u hold one row per interval
 * [t_i, t_{i+1}]; at a point with t_k <= t < t_{k+1} the intervals i < k are integrated over
 * s = t - tau in (t - t_{i+1}, t - t_i) and the current interval k over (0, t - t_k).  Rule and
 * outputs as or_repr. */
int or_repr_nonuniform(const double *verts, int nv, const int32_t *tris, int ne, double alpha,
                       const double *tn, int nt, const double *w, const double *u,
                       const double *pts, int P, int rule_kind, int rule_order, double *sl,
                       double *dl) {
  (void)nv;
  if (nt < 1 || tn[0] != 0.0) return -1;
  for (int k = 0; k < nt; ++k)
    if (!(tn[k + 1] > tn[k])) return -1;
  double lam[3 * 4096], wq[4096];
  int nq = or_triangle_rule(rule_kind, rule_order, lam, wq);
  if (nq <= 0) return -1;
  ld al = (ld)alpha;
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < P; ++p) {
    ld x[3] = {pts[4 * p], pts[4 * p + 1], pts[4 * p + 2]}, t = pts[4 * p + 3];
    int k = 0; /* largest k <= nt with t_k <= t */
    while (k < nt && (ld)tn[k + 1] <= t) ++k;
    ld accs = 0.0L, accd = 0.0L;
    for (int j = 0; j < ne; ++j) {
      tri_t B;
      make_tri(verts, tris + 3 * j, &B);
      for (int q = 0; q < nq; ++q) {
        ld y[3], r[3];
        for (int c = 0; c < 3; ++c) {
          y[c] = lam[3 * q] * B.v[0][c] + lam[3 * q + 1] * B.v[1][c] + lam[3 * q + 2] * B.v[2][c];
          r[c] = x[c] - y[c];
        }
        ld rho = sqrtl(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        ld rn = r[0] * B.n[0] + r[1] * B.n[1] + r[2] * B.n[2];
        ld Wq = wq[q] * B.area;
        ld ws = 0.0L, wd[3] = {0, 0, 0};
        for (int i = 0; i < k; ++i) {
          ld s_lo = t - (ld)tn[i + 1], s_hi = t - (ld)tn[i];
          ws += w[(size_t)i * ne + j] * time_int_G(rho, s_lo, s_hi, al);
          ld gn = time_int_Gn_rn(rho, s_lo, s_hi, al);
          for (int c = 0; c < 3; ++c) wd[c] += u[(size_t)i * nv + tris[3 * j + c]] * gn;
        }
        if (k < nt && t > (ld)tn[k]) {
          ld s_hi = t - (ld)tn[k];
          ws += w[(size_t)k * ne + j] * time_int_G(rho, 0.0L, s_hi, al);
          ld gn = time_int_Gn_rn(rho, 0.0L, s_hi, al);
          for (int c = 0; c < 3; ++c) wd[c] += u[(size_t)k * nv + tris[3 * j + c]] * gn;
        }
        accs += Wq * ws;
        accd += Wq * rn * (lam[3 * q] * wd[0] + lam[3 * q + 1] * wd[1] + lam[3 * q + 2] * wd[2]);
      }
    }
    sl[p] = (double)accs;
    dl[p] = (double)accd;
  }
  return 0;
}

/* ---- vectorised temporal functions for tests (double in/out, long double inside) ---- */
void or_temporal(int which, const double *rho, const double *delta, int n, double alpha,
                 double *out) {
  for (int i = 0; i < n; ++i) {
    ld r = rho[i], d = delta[i], a = alpha, v = 0;
    switch (which) {
      case 0: v = or_g1(r, d, a); break;
      case 1: v = or_F(r, d, a); break;
      case 2: v = or_Fn_rn(r, d, a); break;
      case 3: v = or_g1n_rn(r, d, a); break;
      default: v = NAN;
    }
    out[i] = (double)v;
  }
}

void or_blockfun(int which, const double *rho, const int32_t *d, int n, double h, double alpha,
                 int tmode, double *out) {
  for (int i = 0; i < n; ++i) {
    ld v = which == 0 ? or_Vd(rho[i], d[i], h, alpha, tmode)
         : which == 1 ? or_Kd_rn(rho[i], d[i], h, alpha, tmode)
                      : or_D2d(rho[i], d[i], h, alpha);
    out[i] = (double)v;
  }
}

int or_gauss_legendre01(int n, double *x, double *w) {
  ld gx[64], gw[64];
  if (n < 1 || n > 64) return -1;
  gauss_legendre01(n, gx, gw);
  for (int i = 0; i < n; ++i) { x[i] = (double)gx[i]; w[i] = (double)gw[i]; }
  return n;
}
