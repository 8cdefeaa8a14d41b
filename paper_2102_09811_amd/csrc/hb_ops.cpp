// Entry points beyond assembly: Toeplitz apply, Dirichlet right-hand side, solvers, potentials.
#include <hip/hip_runtime.h>

#include <string>

#include "hb_internal.h"

extern "C" {

int hb_apply(hb_ctx *c, uint32_t op, const double *x, double *y, void *stream) {
  (void)op; (void)x; (void)y; (void)stream;
  if (c) c->err = "hb_apply: not implemented";
  return HB_ESTATE;
}

int hb_rhs_dirichlet(hb_ctx *c, const double *g, double *b, void *stream) {
  (void)g; (void)b; (void)stream;
  if (c) c->err = "hb_rhs_dirichlet: not implemented";
  return HB_ESTATE;
}

int hb_solve(hb_ctx *c, const double *b, double *w, const hb_solve_opts *opts, hb_solve_info *info,
             void *stream) {
  (void)b; (void)w; (void)opts; (void)info; (void)stream;
  if (c) c->err = "hb_solve: not implemented";
  return HB_ESTATE;
}

int hb_eval_repr(hb_ctx *c, const double *pts, int64_t P, const double *w, const double *g,
                 double *u, double *sl, double *dl, void *stream) {
  (void)pts; (void)P; (void)w; (void)g; (void)u; (void)sl; (void)dl; (void)stream;
  if (c) c->err = "hb_eval_repr: not implemented";
  return HB_ESTATE;
}

}  // extern "C"
