"""Error paths and edge cases of the C ABI on a device context.  Every case here is rejected (or
handled) by the library's host-side checks before any kernel is launched."""
import numpy as np
import pytest

from oracle import downstream as ds
from synthetic import cube, tetrahedron

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def test_call_order_and_arguments(torch):
    from paper_2102_09811_amd import (HB_EINVAL, HB_ESTATE, HB_OP_K, HB_OP_V, Context, HBError)
    v, t = tetrahedron()
    ctx = Context(v, t, 1.0, 1.0, 4)
    x = torch.zeros((4, len(t)), dtype=torch.float64, device="cuda")
    with pytest.raises(HBError) as e:          # nothing assembled yet
        ctx.apply(HB_OP_V, x)
    assert e.value.code == HB_ESTATE
    with pytest.raises(HBError) as e:
        ctx.solve(x)
    assert e.value.code == HB_ESTATE
    for ops in (0, 32, 64):
        with pytest.raises(HBError) as e:
            ctx.assemble(ops)
        assert e.value.code == HB_EINVAL
    with pytest.raises(HBError) as e:
        ctx.assemble(HB_OP_V | HB_OP_K, precision=7)
    assert e.value.code == HB_EINVAL
    ctx.assemble()
    with pytest.raises(HBError) as e:          # block range past E_t
        ctx.blocks(HB_OP_V, 3, 2)
    assert e.value.code == HB_EINVAL
    with pytest.raises(HBError) as e:          # no preconditioner installed
        ctx.solve(x + 1.0, precond=True)
    assert e.value.code == HB_ESTATE
    with pytest.raises(HBError) as e:
        ctx.solve(x + 1.0, method=9)
    assert e.value.code == HB_EINVAL
    ctx.close()


def test_gmres_reports_no_convergence(torch):
    from paper_2102_09811_amd import Context
    v, t = cube(2)
    ctx = Context(v, t, 1.0, 1.0, 8)
    ctx.assemble()
    b = torch.from_numpy(np.random.default_rng(3).standard_normal((8, len(t)))).cuda()
    w, info = ctx.solve(b, tol=1e-12, max_iter=3)
    assert not info["converged"] and info["iterations"] == 3
    assert np.isfinite(w.cpu().numpy()).all()
    w, info = ctx.solve(b, tol=1e-8)
    assert info["converged"] and info["rel_residual"] <= 1e-8
    ctx.close()


def test_solve_fallback_and_residual_contract(torch):
    """The plain double GMRES fallback, forced from the host: a preconditioned (or mixed inner)
    phase capped at 2 iterations ends above tol and plain GMRES continues from its iterate.  The
    result meets the tolerance, recomputed here with the oracle's blocks."""
    import oracle
    from paper_2102_09811_amd import Context, HB_SOLVE_GMRES, HB_SOLVE_MIXED_IR
    v, t = cube(2)
    nt = 12
    ctx = Context(v, t, 1.0, 1.0, nt)
    ctx.assemble()
    _, _, y = ctx.precond_spai(exact=True)
    ctx.precond_set(y)
    Vr, _ = oracle.assemble(v, t, 1.0, 1.0, nt)
    bh = np.random.default_rng(4).standard_normal((nt, len(t)))
    b = torch.from_numpy(bh).cuda()
    for method in (HB_SOLVE_GMRES, HB_SOLVE_MIXED_IR):
        w, info = ctx.solve(b, method=method, tol=1e-8, precond=True, precond_max_iter=2)
        res = np.linalg.norm(bh - ds.toeplitz_apply(Vr, w.cpu().numpy())) / np.linalg.norm(bh)
        print("[gpu-test] method %d capped: it=%d fallback=%s restarts=%d res=%.2e (oracle %.2e)" % (
            method, info["iterations"], info["fallback"], info["restarts"], info["rel_residual"],
            res), flush=True)
        assert info["fallback"] and info["converged"] and info["rel_residual"] <= 1e-8
        assert res <= 1.01e-8
        w, info = ctx.solve(b, method=method, tol=1e-8, precond=True)
        assert not info["fallback"] and info["converged"] and info["rel_residual"] <= 1e-8
    ctx.close()


def test_time_limits(torch):
    """E_t = 300: assembly works; the Toeplitz product (and so every solver) refuses E_t > 256;
    potentials still work.  E_t = 2000: the potentials refuse (their per-interval table, 12
    doubles per interval, no longer fits in one workgroup's LDS)."""
    from paper_2102_09811_amd import HB_EINVAL, HB_OP_V, Context, HBError
    v, t = tetrahedron()
    ctx = Context(v, t, 1.0, 1.0, 300)
    ctx.assemble()
    x = torch.zeros((300, len(t)), dtype=torch.float64, device="cuda")
    with pytest.raises(HBError) as e:
        ctx.apply(HB_OP_V, x)
    assert e.value.code == HB_EINVAL
    with pytest.raises(HBError) as e:
        ctx.solve(x + 1.0)
    assert e.value.code == HB_EINVAL
    pts = torch.tensor([[0.1, 0.1, 0.1, 0.5]], dtype=torch.float64, device="cuda")
    g = torch.zeros((300, len(v)), dtype=torch.float64, device="cuda")
    u = ctx.eval_repr(pts, x, g)
    assert float(u.abs().max()) == 0.0
    empty = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    assert ctx.eval_repr(empty, x, g).numel() == 0
    ctx.close()
    ctx = Context(v, t, 1.0, 1.0, 2000)
    x = torch.zeros((2000, len(t)), dtype=torch.float64, device="cuda")
    g = torch.zeros((2000, len(v)), dtype=torch.float64, device="cuda")
    with pytest.raises(HBError) as e:
        ctx.eval_repr(pts, x, g)
    assert e.value.code == HB_EINVAL
    ctx.close()


def test_neumann_call_order_and_arguments(torch):
    from paper_2102_09811_amd import (HB_EINVAL, HB_ESTATE, HB_OP_D, HB_OP_K, HB_OP_KT, HB_OP_V,
                                      HB_SOLVE_TIMEMARCH, Context, HBError)
    v, t = tetrahedron()
    ctx = Context(v, t, 1.0, 1.0, 4)
    psi = torch.zeros((4, len(t)), dtype=torch.float64, device="cuda")
    b = torch.zeros((4, len(v)), dtype=torch.float64, device="cuda")
    for call in (lambda: ctx.rhs_neumann(psi), lambda: ctx.solve_neumann(b),
                 lambda: ctx.apply(HB_OP_D, b), lambda: ctx.apply(HB_OP_KT, psi),
                 lambda: ctx.assemble(HB_OP_D)):
        with pytest.raises(HBError) as e:
            call()
        assert e.value.code == HB_ESTATE
    with pytest.raises(HBError) as e:
        ctx.assemble(32)
    assert e.value.code == HB_EINVAL
    ctx.assemble(HB_OP_V | HB_OP_K | HB_OP_D)
    from paper_2102_09811_amd import binding
    import ctypes
    o = binding.SolveOpts()
    o.method, o.tol, o.max_iter = HB_SOLVE_TIMEMARCH, 1e-8, 10
    info = binding.SolveInfo()
    u = torch.zeros_like(b)
    rc = binding.lib().hb_solve_neumann(ctx._h, binding._ptr(b + 1.0), binding._ptr(u), ctypes.byref(o),
                                        ctypes.byref(info), None)
    assert rc == HB_EINVAL
    u, info = ctx.solve_neumann(b)       # zero right-hand side: zero solution, no iterations
    assert info["converged"] and float(u.abs().max()) == 0.0
    ctx.close()


def test_measure_peaks(torch):
    """The vector-ALU microbenchmarks return rates of the right order: at most the published
    MI355X figures (FP64 78.6, FP32 157.3 TFLOP/s) plus measurement slack, and clearly nonzero."""
    from paper_2102_09811_amd import measure_peaks
    p = measure_peaks()
    print("[gpu-test] measured peaks: %s" % p, flush=True)
    assert 10.0 < p["fp64_fma_tflops"] < 1.1 * 78.6
    assert 10.0 < p["fp32_fma_tflops"] < 1.1 * 157.3
    assert 100.0 < p["fp64_rsq_gops"] < 1.1 * 78.6e3 / 2
