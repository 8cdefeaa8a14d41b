"""hb_apply_noalloc (the block-Toeplitz product with the library's fixed scratch) against hb_apply
on the same assembled blocks, through the C ABI.

Both entry points run the same kernels; the fixed scratch may force a narrower split of the
product (fewer partial results), which changes only the order in which the partial sums are
added.  Bar: max |y_noalloc - y| <= 1e-14 max |y| (double blocks), 1e-6 (float blocks, whose
partial sums are float).  Two calls in a row, the second on a smaller context, check that nothing
of the first call's scratch contents leaks into the second.
"""
import sys

import numpy as np
import pytest

from synthetic import cube, icosphere

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    _t.cuda.set_device(0)
    return _t


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _compare(torch, ctx, op, rows_in, rows_out, bar, seed):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(ctx.n_t, rows_in, dtype=torch.float64, device="cuda", generator=gen)
    y_ref = ctx.apply(op, x)
    y = torch.full((ctx.n_t, rows_out), float("nan"), dtype=torch.float64, device="cuda")
    ctx.apply_noalloc(op, x, y)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    e = _rel(y, y_ref)
    say("  op %d: max |y_noalloc - y| / max |y| = %.2e" % (op, e))
    assert e <= bar


def test_noalloc_apply_matches_apply_two_calls(torch):
    from paper_2102_09811_amd import HB_OP_K, HB_OP_KT, HB_OP_V, Context
    # first call: 768 panels x 128 steps, where the fixed scratch narrows the split of V and K
    v, t = cube(8)
    say("no-alloc apply: cube(8) %d panels, 128 steps (split narrowed to the scratch)" % len(t))
    ctx = Context(v, t, 1.0, 1.0, 128)
    ctx.assemble(HB_OP_V | HB_OP_K)
    _compare(torch, ctx, HB_OP_V, ctx.n_tris, ctx.n_tris, 1e-14, 1)
    _compare(torch, ctx, HB_OP_K, ctx.n_verts, ctx.n_tris, 1e-14, 2)
    ctx.close()
    # second call: a smaller context (48 panels, 8 steps) on the same scratch
    v, t = cube(2)
    say("no-alloc apply: cube(2) %d panels, 8 steps" % len(t))
    ctx = Context(v, t, 0.7, 1.0, 8)
    ctx.assemble(HB_OP_V | HB_OP_K)
    _compare(torch, ctx, HB_OP_V, ctx.n_tris, ctx.n_tris, 1e-14, 3)
    _compare(torch, ctx, HB_OP_K, ctx.n_verts, ctx.n_tris, 1e-14, 4)
    # K_h^T: only after hb_apply has formed the transposed blocks
    x = torch.ones(ctx.n_t, ctx.n_tris, dtype=torch.float64, device="cuda")
    y = torch.empty(ctx.n_t, ctx.n_verts, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception) as ei:
        ctx.apply_noalloc(HB_OP_KT, x, y)
    assert getattr(ei.value, "code", None) == -7
    _compare(torch, ctx, HB_OP_KT, ctx.n_tris, ctx.n_verts, 1e-14, 5)
    ctx.close()


def test_noalloc_apply_float_storage(torch):
    from paper_2102_09811_amd import HB_DTYPE_F32, HB_OP_K, HB_OP_V, Context
    v, t = cube(4)
    say("no-alloc apply: cube(4), float block storage, 40 steps")
    ctx = Context(v, t, 1.0, 1.0, 40, storage=HB_DTYPE_F32)
    ctx.assemble(HB_OP_V | HB_OP_K)
    _compare(torch, ctx, HB_OP_V, ctx.n_tris, ctx.n_tris, 1e-6, 6)
    _compare(torch, ctx, HB_OP_K, ctx.n_verts, ctx.n_tris, 1e-6, 7)
    ctx.close()


def test_noalloc_apply_rejects_oversize(torch):
    """E_t x E_x x 8 bytes above 32 MiB is rejected before any state check or launch."""
    from paper_2102_09811_amd import HB_OP_V, Context
    v, t = icosphere(5)  # 20480 panels: 256 x 20480 x 8 B = 40 MiB of partial results
    say("no-alloc apply: oversize rejection (icosphere(5), 256 steps, not assembled)")
    ctx = Context(v, t, 1.0, 1.0, 256)
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception) as ei:
        ctx.apply_noalloc(HB_OP_V, x, x)
    assert getattr(ei.value, "code", None) == -1
    ctx.close()
