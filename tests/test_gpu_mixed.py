"""Mixed precision (float separated pairs at large d, float-MFMA apply, iterative refinement)
against the oracle and against the double path.

Bars: per-block max error relative to the block's max <= 1e-6 for every d, V and K, of the mixed
assembly against the oracle (every row of the 192-triangle cube, sampled rows of the
1280-triangle sphere; the 3072-triangle cube's sampled rows are in the assembly tests) and against
the double assembly (the error the mixed path adds, reported per block); the refinement solve
reaches ||b - V_h w|| / ||b|| <= 1e-8 with the double operator.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import downstream as ds
from synthetic import cube, exp_solution, icosphere, nodal_samples

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


def per_block_rel(A, B):
    """max |A^d - B^d| / max |A^d| per block, on the device."""
    import torch
    num = (A - B).abs().reshape(A.shape[0], -1).amax(1)
    den = A.abs().reshape(A.shape[0], -1).amax(1)
    return (num / den).cpu().numpy()


@pytest.mark.parametrize("mesh,nt,alpha,dmin", [("cube4", 16, 1.0, None), ("cube4", 40, 0.5, None),
                                                ("icosphere3", 64, 1.0, None),
                                                ("cube4", 40, 1.0, 8)])
def test_mixed_assembly_per_block(mesh, nt, alpha, dmin):
    """Float separated pairs from the first Taylor block (d = 3, or the option mixed_d_min = 8):
    every block within 1e-6 of the double assembly and of the oracle; the closed-form blocks stay
    identical to the double assembly."""
    import torch
    from paper_2102_09811_amd import Context, HB_OP_K, HB_OP_V, HB_PREC_MIXED
    v, t = cube(4) if mesh == "cube4" else icosphere(3)
    say("mixed assembly %s nt=%d alpha=%g mixed_d_min=%s" % (mesh, nt, alpha, dmin))
    opts = {} if dmin is None else {"mixed_d_min": dmin}
    ctx = Context(v, t, alpha, 1.0, nt, **opts)
    ctx.assemble()
    V64, K64 = ctx.blocks(HB_OP_V), ctx.blocks(HB_OP_K)
    ctx.assemble(precision=HB_PREC_MIXED)
    Vm, Km = ctx.blocks(HB_OP_V), ctx.blocks(HB_OP_K)
    eV, eK = per_block_rel(V64, Vm), per_block_rel(K64, Km)
    d0 = 3 if dmin is None else dmin                     # first float block
    say("max e_V=%.2e max e_K=%.2e; first float block %d" % (eV.max(), eK.max(), d0))
    assert eV.max() <= 1e-6 and eK.max() <= 1e-6
    assert np.all(eV[:min(d0, nt)] == 0.0)              # double blocks unchanged
    assert np.all(eK[:min(d0, nt)] <= 1e-14)            # (K by atomics: summation order)
    if nt > d0:
        assert eV[d0:].max() > 0.0                       # the float path was taken
    # against the oracle: every row of the cube, 8 rows of the sphere
    rows = np.arange(len(t)) if mesh == "cube4" else np.linspace(0, len(t) - 1, 8).astype(np.int64)
    Vr, Kr = oracle.assemble(v, t, alpha, 1.0, nt, rows=rows.astype(np.int32))
    rt = torch.from_numpy(rows).cuda()
    oV = ds.block_rel_error(Vr, Vm[:, rt].cpu().numpy())
    oK = ds.block_rel_error(Kr, Km[:, rt].cpu().numpy())
    say("against the oracle (%d rows): max e_V=%.2e max e_K=%.2e" % (len(rows), oV.max(), oK.max()))
    assert oV.max() <= 1e-6 and oK.max() <= 1e-6
    ctx.close()


def test_float_apply_and_refinement_solve():
    import torch
    from paper_2102_09811_amd import Context, HB_OP_V, HB_SOLVE_GMRES, HB_SOLVE_MIXED_IR
    v, t = icosphere(3)
    nt = 64
    say("float apply / refinement on icosphere3 nt=64")
    ctx = Context(v, t, 1.0, 1.0, nt)
    ctx.assemble()
    g = nodal_samples(v, nt, 1.0, lambda x, tt: exp_solution(x, tt, 1.0))
    gd = torch.from_numpy(g).cuda()
    b = ctx.rhs_dirichlet(gd)
    w64, i64 = ctx.solve(b, method=HB_SOLVE_GMRES, tol=1e-8)
    wm, im = ctx.solve(b, method=HB_SOLVE_MIXED_IR, tol=1e-8)
    say("gmres: it=%d res=%.2e %.1f ms | mixed: it=%d ref=%d res=%.2e %.1f ms" % (
        i64["iterations"], i64["rel_residual"], 1e3 * i64["seconds"], im["iterations"],
        im["refinements"], im["rel_residual"], 1e3 * im["seconds"]))
    assert im["converged"] and im["rel_residual"] <= 1e-8
    rel = float((wm - w64).norm() / w64.norm())
    assert rel <= 1e-5, rel
    ctx.close()


def test_cube3072_nt128_mixed_error():
    """3072-triangle cube, 128 steps, alpha in {0.5, 1, 2}: mixed vs double per-block error."""
    from paper_2102_09811_amd import Context, HB_OP_K, HB_OP_V, HB_PREC_MIXED
    v, t = cube(16)
    for alpha in (0.5, 1.0, 2.0):
        say("cube16 nt=128 alpha=%g" % alpha)
        ctx = Context(v, t, alpha, 1.0, 128)
        worst = {}
        for op in (HB_OP_V, HB_OP_K):
            ctx.assemble(op)
            ref = ctx.blocks(op)
            ctx.assemble(op, precision=HB_PREC_MIXED)
            e = per_block_rel(ref, ctx.blocks(op))
            del ref
            worst[op] = e
        say("alpha=%g: max e_V=%.2e (d=%d) max e_K=%.2e (d=%d)" % (
            alpha, worst[HB_OP_V].max(), worst[HB_OP_V].argmax(), worst[HB_OP_K].max(),
            worst[HB_OP_K].argmax()))
        assert worst[HB_OP_V].max() <= 1e-6 and worst[HB_OP_K].max() <= 1e-6
        ctx.close()
        import torch
        torch.cuda.empty_cache()
