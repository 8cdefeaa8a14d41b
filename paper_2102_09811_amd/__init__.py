"""MI355X (gfx950) space-time boundary element method for the 3D heat equation.

Semi-analytic assembly of the block-Toeplitz single- and double-layer matrices, block-Toeplitz
apply, Dirichlet solves, the hypersingular operator and Neumann solves, and the representation
formula (arXiv 2102.09811), as hand-written HIP
kernels behind the C ABI in include/heatbem.h.  ``binding`` marshals arguments to that library.
"""
from .binding import (Context, NonuniformContext, HBError, PCNet, check_mesh, lib, measure_peaks, precond_train, HB_OP_V, HB_OP_K, HB_OP_D, HB_OP_KT,
                      HB_OP_V11, HB_PREC_FP64,
                      HB_PREC_MIXED, HB_DTYPE_F64, HB_DTYPE_F32, HB_SOLVE_GMRES,
                      HB_SOLVE_TIMEMARCH, HB_SOLVE_MIXED_IR, HB_OK, HB_EINVAL, HB_EMESH,
                      HB_EORIENT, HB_ENOMEM, HB_EHIP, HB_ENOCONV, HB_ESTATE)

__all__ = ["Context", "NonuniformContext", "HBError", "PCNet", "check_mesh", "lib", "measure_peaks", "precond_train", "HB_OP_V", "HB_OP_K", "HB_OP_D", "HB_OP_KT",
           "HB_OP_V11", "HB_PREC_FP64",
           "HB_PREC_MIXED", "HB_DTYPE_F64", "HB_DTYPE_F32", "HB_SOLVE_GMRES",
           "HB_SOLVE_TIMEMARCH", "HB_SOLVE_MIXED_IR", "HB_OK", "HB_EINVAL", "HB_EMESH",
           "HB_EORIENT", "HB_ENOMEM", "HB_EHIP", "HB_ENOCONV", "HB_ESTATE"]
