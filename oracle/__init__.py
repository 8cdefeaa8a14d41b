"""Oracle for the space-time heat BEM (arXiv 2102.09811) -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU implementation of everything the HIP path computes.  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import it.
It shares no code with ``paper_2102_09811_amd`` and does not import it.

* ``oracle.c`` (long double, OpenMP): temporal antiderivatives, triangle and Sauter-Schwab rules,
  pair classification, block assembly (direct and the paper's i_t order), representation formula,
  the second part D_h^2 of the hypersingular operator, the p1 single layer V_h^{11}; and a
  plain double-precision assembly in the paper's level order (``assemble_plain``), the timed
  CPU baseline; blocks on non-uniform time grids (``assemble_nonuniform``).
* ``downstream.py`` (numpy/scipy, float64): mass matrices, L2 projections, block-Toeplitz apply,
  right-hand sides (Dirichlet and Neumann), D_h^1 from V_h by the surface curls, time marching,
  GMRES, L2 / l2 errors.
"""
from .core import (lib, build, temporal, blockfun, triangle_rule, ss_rule, gauss_legendre01,
                   pair_points, assemble, assemble_plain, assemble_nonuniform, nu_blockfun, assemble_d2, assemble_v11, pair_blocks, repr_eval,
                   repr_eval_nonuniform)
from . import downstream

__all__ = ["lib", "build", "temporal", "blockfun", "triangle_rule", "ss_rule",
           "gauss_legendre01", "pair_points", "assemble", "assemble_plain", "assemble_nonuniform", "nu_blockfun", "assemble_d2", "assemble_v11", "pair_blocks", "repr_eval", "repr_eval_nonuniform", "downstream"]
