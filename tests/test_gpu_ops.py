"""GPU parity of the block-Toeplitz apply, the Dirichlet right-hand side, the solvers and the
representation formula against the oracle (through the C ABI).

Bars: apply on identical blocks agrees with the oracle's apply to 1e-14 (relative to max|y|);
against the oracle's own blocks to 1e-11; solves reach ||b - V_h w|| / ||b|| <= 1e-8 measured
with the oracle's blocks; the potentials agree with the long-double oracle to 1e-11 relative
to max|u|; the Dirichlet pipeline reproduces the paper's Table 6.1 first level.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import downstream as ds
from synthetic import (ExactSolution, ball_points, box_points, cube, exp_solution, icosphere,
                       nodal_samples, space_time_points)

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.fixture(scope="module")
def c1(torch):
    """192-triangle unit cube, alpha = 1, T = 1, 16 steps: context + oracle blocks."""
    from paper_2102_09811_amd import Context
    v, t = cube(4)
    Vr, Kr = oracle.assemble(v, t, 1.0, 1.0, 16)
    say("c1 context")
    ctx = Context(v, t, 1.0, 1.0, 16)
    ctx.assemble()
    return v, t, ctx, Vr, Kr


@pytest.mark.parametrize("nt", [16, 70])
def test_apply_matches_oracle(torch, nt):
    from paper_2102_09811_amd import Context, HB_OP_K, HB_OP_V
    v, t = cube(4)
    Vr, Kr = oracle.assemble(v, t, 0.8, 1.0, nt)
    say("apply cube4 nt=%d" % nt)
    ctx = Context(v, t, 0.8, 1.0, nt)
    ctx.assemble()
    Vg, Kg = ctx.blocks(HB_OP_V, device=False), ctx.blocks(HB_OP_K, device=False)
    rng = np.random.default_rng(nt)
    for op, Ag, Ar, cols in ((HB_OP_V, Vg, Vr, len(t)), (HB_OP_K, Kg, Kr, len(v))):
        x = rng.standard_normal((nt, cols))
        y = ctx.apply(op, torch.from_numpy(x).cuda()).cpu().numpy()
        assert rel_inf(y, ds.toeplitz_apply(Ag, x)) <= 1e-14
        assert rel_inf(y, ds.toeplitz_apply(Ar, x)) <= 1e-11
    ctx.close()


def test_apply_full_size(torch):
    """1280 triangles x 64 steps: apply of V and K against numpy on the same device blocks."""
    from paper_2102_09811_amd import Context, HB_OP_K, HB_OP_V
    v, t = icosphere(3)
    say("apply icosphere3 nt=64")
    ctx = Context(v, t, 1.0, 1.0, 64)
    ctx.assemble()
    rng = np.random.default_rng(5)
    for op, cols in ((HB_OP_V, len(t)), (HB_OP_K, len(v))):
        A = ctx.blocks(op, device=False)
        x = rng.standard_normal((64, cols))
        y = ctx.apply(op, torch.from_numpy(x).cuda()).cpu().numpy()
        assert rel_inf(y, ds.toeplitz_apply(A, x)) <= 1e-14
    ctx.close()


def test_rhs_matches_oracle(torch, c1):
    v, t, ctx, Vr, Kr = c1
    g = nodal_samples(v, 16, 1.0, lambda x, tt: exp_solution(x, tt, 1.0))
    say("rhs c1")
    b = ctx.rhs_dirichlet(torch.from_numpy(g).cuda()).cpu().numpy()
    ref = ds.rhs_dirichlet(Kr, ds.mass_p0p1(v, t), g, 1.0 / 16)
    assert rel_inf(b, ref) <= 1e-11


@pytest.mark.parametrize("method", [0, 1])
def test_solvers_reach_tolerance(torch, c1, method):
    from paper_2102_09811_amd import HB_SOLVE_GMRES
    v, t, ctx, Vr, Kr = c1
    g = nodal_samples(v, 16, 1.0, lambda x, tt: exp_solution(x, tt, 1.0))
    b = ds.rhs_dirichlet(Kr, ds.mass_p0p1(v, t), g, 1.0 / 16)
    say("solve c1 method=%d" % method)
    w, info = ctx.solve(torch.from_numpy(b).cuda(), method=method, tol=1e-8)
    w = w.cpu().numpy()
    res = np.linalg.norm(b - ds.toeplitz_apply(Vr, w)) / np.linalg.norm(b)
    say("solve c1 method=%d: it=%d res(device)=%.2e res(oracle blocks)=%.2e" %
        (method, info["iterations"], info["rel_residual"], res))
    assert info["converged"]
    assert info["rel_residual"] <= 1e-8 and res <= 1.1e-8
    wr = ds.time_march(Vr, b)
    if method == 1:   # direct: agrees with the oracle's Cholesky time marching
        assert rel_inf(w, wr) <= 1e-10
    else:             # iterative: solutions agree within cond(V_h) x tolerance
        nt, ne = Vr.shape[0], Vr.shape[1]
        full = np.zeros((nt * ne, nt * ne))
        for k in range(nt):
            for d in range(k + 1):
                full[k * ne:(k + 1) * ne, (k - d) * ne:(k - d + 1) * ne] = Vr[d]
        cond = np.linalg.cond(full)
        diff = np.linalg.norm(w - wr) / np.linalg.norm(wr)
        say("cond(V_h) = %.3e, solution difference (2-norm) %.3e" % (cond, diff))
        assert diff <= 2 * cond * 1e-8
    if method == HB_SOLVE_GMRES:
        assert info["iterations"] > 3


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_time_marching_long(torch, storage):
    """E_t = 70 (halved down to runs of at most 4 steps, uneven halves): time marching against
    the oracle's LU time marching on the same blocks, double and float block storage."""
    from paper_2102_09811_amd import Context, HB_DTYPE_F32, HB_OP_V, HB_SOLVE_TIMEMARCH
    v, t = cube(2)
    nt = 70
    opts = {"storage": HB_DTYPE_F32} if storage == "f32" else {}
    say("time marching cube2 nt=%d storage=%s" % (nt, storage))
    ctx = Context(v, t, 0.7, 1.0, nt, **opts)
    ctx.assemble()
    Vg = ctx.blocks(HB_OP_V, device=False).astype(np.float64)
    rng = np.random.default_rng(21)
    b = rng.standard_normal((nt, len(t)))
    bd = torch.from_numpy(b).cuda()
    tol = 1e-12 if storage == "f64" else 1e-5
    w, info = ctx.solve(bd, method=HB_SOLVE_TIMEMARCH, tol=tol)
    w = w.cpu().numpy()
    wr = ds.time_march(Vg, b)
    say("time marching %s: rel diff %.2e, residual %.2e" % (storage, rel_inf(w, wr), info["rel_residual"]))
    assert info["converged"] and info["rel_residual"] <= tol
    # float storage: the history products run on float MFMA (sources rounded to float)
    assert rel_inf(w, wr) <= (1e-10 if storage == "f64" else 1e-5)
    res = np.linalg.norm(b - ds.toeplitz_apply(Vg, w)) / np.linalg.norm(b)
    assert res <= (1e-12 if storage == "f64" else 1e-5), res
    if storage == "f32":
        # the residual of float blocks (sources rounded to float) cannot certify 1e-12: three
        # repeated forward substitutions on the residual, then HB_ENOCONV
        _, info = ctx.solve(bd, method=HB_SOLVE_TIMEMARCH, tol=1e-12)
        assert not info["converged"] and info["restarts"] == 3 and info["rel_residual"] > 1e-12
    ctx.close()


def test_repr_matches_oracle(torch, c1):
    v, t, ctx, Vr, Kr = c1
    rng = np.random.default_rng(11)
    w = rng.standard_normal((16, len(t)))
    g = rng.standard_normal((16, len(v)))
    pts = space_time_points(box_points(300, 0.2, 0.8, seed=3), 0.0, 1.0, seed=3)
    pts[:5, 3] = [0.0, 1.0, 0.5, 1.0 / 16, 0.999]   # t on grid points, T, t = 0
    say("repr c1 P=%d" % len(pts))
    u, sl, dl = ctx.eval_repr(torch.from_numpy(pts).cuda(), torch.from_numpy(w).cuda(),
                              torch.from_numpy(g).cuda(), parts=True)
    slr, dlr = oracle.repr_eval(v, t, 1.0, 1.0, 16, w, g, pts)
    assert rel_inf(sl.cpu().numpy(), slr) <= 1e-11
    assert rel_inf(dl.cpu().numpy(), dlr) <= 1e-11
    assert rel_inf(u.cpu().numpy(), slr - dlr) <= 1e-11


@pytest.mark.parametrize("alpha", [0.3, 2.0])
def test_repr_long_history(torch, alpha):
    """E_t = 70: every interval-distance class of the potential evaluation (closed form near the
    point's time, Taylor polynomials of degree 20 .. 8 further back), t anywhere in (0, T]."""
    from paper_2102_09811_amd import Context
    v, t = cube(2)
    nt = 70
    rng = np.random.default_rng(5)
    w = rng.standard_normal((nt, len(t)))
    g = rng.standard_normal((nt, len(v)))
    pts = space_time_points(box_points(160, 0.1, 0.9, seed=6), 0.0, 1.0, seed=6)
    pts[:4, 3] = [1.0, 0.5, 3.0 / nt, 2.5 / nt]
    say("repr long history alpha=%g P=%d" % (alpha, len(pts)))
    ctx = Context(v, t, alpha, 1.0, nt)
    u, sl, dl = ctx.eval_repr(torch.from_numpy(pts).cuda(), torch.from_numpy(w).cuda(),
                              torch.from_numpy(g).cuda(), parts=True)
    slr, dlr = oracle.repr_eval(v, t, alpha, 1.0, nt, w, g, pts)
    assert rel_inf(sl.cpu().numpy(), slr) <= 1e-11
    assert rel_inf(dl.cpu().numpy(), dlr) <= 1e-11
    assert rel_inf(u.cpu().numpy(), slr - dlr) <= 1e-11


def test_repr_full_size_sampled(torch):
    """The benchmarked potential evaluation (1280-triangle sphere, 64 steps, points in the ball of
    radius 0.5 with t in [0.25, 0.75]) on 48 of its points against the oracle."""
    from paper_2102_09811_amd import Context
    v, t = icosphere(3)
    nt = 64
    rng = np.random.default_rng(8)
    w = rng.standard_normal((nt, len(t)))
    g = rng.standard_normal((nt, len(v)))
    pts = space_time_points(ball_points(10000, 0.5, seed=0), 0.25, 0.75, seed=0)[::208][:48]
    say("repr icosphere3 nt=64 P=%d" % len(pts))
    ctx = Context(v, t, 1.0, 1.0, nt)
    u, sl, dl = ctx.eval_repr(torch.from_numpy(np.ascontiguousarray(pts)).cuda(),
                              torch.from_numpy(w).cuda(), torch.from_numpy(g).cuda(), parts=True)
    slr, dlr = oracle.repr_eval(v, t, 1.0, 1.0, nt, w, g, pts)
    assert rel_inf(sl.cpu().numpy(), slr) <= 1e-11
    assert rel_inf(dl.cpu().numpy(), dlr) <= 1e-11


def test_dirichlet_pipeline_table61(torch):
    """The paper's convergence problem on its coarsest mesh (192 triangles, 8 steps, alpha 0.5):
    GPU assembly + right-hand side + GMRES + potentials."""
    from paper_2102_09811_amd import Context
    alpha, T, nt = 0.5, 1.0, 8
    ex = ExactSolution(alpha, (0.0, 0.0, 1.5))
    v, t = cube(4, -1.0, 1.0)
    g = ds.project_p1p0(v, t, nt, T, ex.u)
    pts = space_time_points(box_points(2000, -0.5, 0.5, seed=0), 0.25, 0.75, seed=0)
    say("dirichlet pipeline 192/8")
    ctx = Context(v, t, alpha, T, nt)
    ctx.assemble()
    gd = torch.from_numpy(g).cuda()
    b = ctx.rhs_dirichlet(gd)
    w, info = ctx.solve(b, tol=1e-8)
    u = ctx.eval_repr(torch.from_numpy(pts).cuda(), w, gd).cpu().numpy()
    w = w.cpu().numpy()
    e_w = ds.l2_error_p0(v, t, nt, T, w, lambda x, n, tt: ex.flux(x, n, tt))
    e_r = ds.relative_l2(ex.u(pts[:, :3], pts[:, 3]), u)
    say("pipeline: L2(w)=%.3e l2(repr)=%.3e it=%d" % (e_w, e_r, info["iterations"]))
    assert abs(e_w / 6.07e-1 - 1) < 0.05 and abs(e_r / 2.99e-2 - 1) < 0.25
    ctx.close()
