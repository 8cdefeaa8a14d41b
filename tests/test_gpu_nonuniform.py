"""GPU parity of the non-uniform time-step path (the paper's outlook, Sec. 7, with the block
integrals of Sec. 3.1 and 3.2 at general interval endpoints) against the oracle, through the C ABI.

* blocks V^{k,i}, K^{k,i} (all 0 <= i <= k < E_t) on graded grids: block-relative <= 1e-12 against
  the oracle's long-double assembly (four-term difference, trapezoid-weighted Gauss where it would
  cancel) -- the GPU takes the four-term difference or the even Taylor series of the trapezoid
  weight, an independent evaluation of the same integral;
* a uniform grid through this path reproduces the oracle's Toeplitz blocks V^{k-i}, K^{k-i};
* the block lower-triangular product, the right-hand side (1/2 M_h + K_h) g with
  M_h = blockdiag(h_k M_x), GMRES to 1e-8 and time marching (inverses of every V^{k,k}) against
  numpy on the oracle's blocks;
* the potentials (Sec. 3.5 over general intervals) against the oracle's closed forms;
* the entry points that a non-uniform context does not support return HB_EINVAL.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import downstream as ds
from synthetic import cube, octahedron

pytestmark = pytest.mark.gpu

GRID = np.array([0.0, 0.05, 0.12, 0.2, 0.33, 0.45, 0.6, 0.72, 0.9, 1.0])  # irregular, 9 steps


def graded(n, gamma):
    return (np.arange(n + 1) / n) ** gamma


def geometric(n, q, T=1.0):
    h = q ** np.arange(n)
    return np.concatenate([[0.0], np.cumsum(h)]) * (T / h.sum())


def say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def block_errors(A, R):
    """max over blocks of max |A - R| / max |R| (blocks with R == 0 compared absolutely)."""
    num = np.abs(A - R).reshape(len(R), -1).max(axis=1)
    den = np.abs(R).reshape(len(R), -1).max(axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


CASES = {
    "octa_irregular9": (octahedron, GRID, 0.7, None, 4),
    "cube2_graded12": (lambda: cube(2), graded(12, 1.6), 1.0, np.array([0, 5, 11, 17, 23, 30, 41, 47]), 4),
    "cube2_geometric16_ss3": (lambda: cube(2), geometric(16, 1.18), 0.5, np.array([2, 19, 36]), 3),
    "cube4_graded10": (lambda: cube(4), graded(10, 2.0), 2.0, np.array([0, 63, 101, 191]), 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_nu_blocks_match_oracle(torch, case):
    from paper_2102_09811_amd import HB_OP_K, HB_OP_V, NonuniformContext
    mesh, tn, alpha, rows, ss = CASES[case]
    v, t = mesh()
    rows = np.arange(len(t)) if rows is None else rows
    say("nonuniform blocks %s: %d panels, %d steps, %d rows" % (case, len(t), len(tn) - 1, len(rows)))
    Vr, Kr = oracle.assemble_nonuniform(v, t, alpha, tn, rows=rows, ss_order=ss)
    ctx = NonuniformContext(v, t, alpha, tn, ss_order=ss)
    ctx.assemble(HB_OP_V | HB_OP_K)
    V = ctx.blocks(HB_OP_V, device=False)[:, rows, :]
    K = ctx.blocks(HB_OP_K, device=False)[:, rows, :]
    ctx.close()
    eV, eK = block_errors(V, Vr), block_errors(K, Kr)
    say("  max block-relative error V %.2e (block %d), K %.2e (block %d)"
        % (eV.max(), eV.argmax(), eK.max(), eK.argmax()))
    assert eV.max() <= 1e-12 and eK.max() <= 1e-12


def test_nu_uniform_grid_reproduces_toeplitz(torch):
    from paper_2102_09811_amd import HB_OP_K, HB_OP_V, NonuniformContext
    v, t = cube(2)
    nt, alpha = 20, 0.8
    say("nonuniform path on a uniform grid: cube(2), %d steps" % nt)
    Vr, Kr = oracle.assemble(v, t, alpha, 1.0, nt)
    ctx = NonuniformContext(v, t, alpha, np.linspace(0.0, 1.0, nt + 1))
    ctx.assemble(HB_OP_V | HB_OP_K)
    V = ctx.blocks(HB_OP_V, device=False)
    K = ctx.blocks(HB_OP_K, device=False)
    ctx.close()
    idx = [(k, i) for k in range(nt) for i in range(k + 1)]
    eV = block_errors(V, np.stack([Vr[k - i] for k, i in idx]))
    eK = block_errors(K, np.stack([Kr[k - i] for k, i in idx]))
    say("  against the Toeplitz blocks: V %.2e, K %.2e" % (eV.max(), eK.max()))
    assert eV.max() <= 1e-12 and eK.max() <= 1e-12


def test_nu_apply_rhs_and_solve(torch):
    from paper_2102_09811_amd import HB_OP_K, HB_OP_V, HB_SOLVE_TIMEMARCH, NonuniformContext
    v, t = octahedron()
    tn, alpha = GRID, 0.7
    nt, ne, nv = len(tn) - 1, len(t), len(v)
    say("nonuniform apply / rhs / GMRES: octahedron, 9 irregular steps")
    Vr, Kr = oracle.assemble_nonuniform(v, t, alpha, tn)
    ctx = NonuniformContext(v, t, alpha, tn)
    ctx.assemble(HB_OP_V | HB_OP_K)

    def tri_apply(B, x):
        y = np.zeros((nt, B.shape[1]))
        for k in range(nt):
            for i in range(k + 1):
                y[k] += B[k * (k + 1) // 2 + i] @ x[i]
        return y

    rng = np.random.default_rng(3)
    x = rng.standard_normal((nt, ne))
    xg = rng.standard_normal((nt, nv))
    y = ctx.apply(HB_OP_V, torch.from_numpy(x).cuda()).cpu().numpy()
    yk = ctx.apply(HB_OP_K, torch.from_numpy(xg).cuda()).cpu().numpy()
    yr, ykr = tri_apply(Vr, x), tri_apply(Kr, xg)
    e1 = np.abs(y - yr).max() / np.abs(yr).max()
    e2 = np.abs(yk - ykr).max() / np.abs(ykr).max()
    # data: exp(alpha t + x.e) sampled at the vertices and interval midpoints
    tm = 0.5 * (tn[1:] + tn[:-1])
    e = np.ones(3) / np.sqrt(3.0)
    g = np.exp(alpha * tm[:, None] + (v @ e)[None, :])
    b = ctx.rhs_dirichlet(torch.from_numpy(g).cuda()).cpu().numpy()
    M = ds.mass_p0p1(v, t)
    br = tri_apply(Kr, g) + 0.5 * (tn[1:] - tn[:-1])[:, None] * (M @ g.T).T
    e3 = np.abs(b - br).max() / np.abs(br).max()
    w, info = ctx.solve(torch.from_numpy(br).cuda(), tol=1e-8)
    w = w.cpu().numpy()
    res = np.linalg.norm(br - tri_apply(Vr, w)) / np.linalg.norm(br)
    # block forward substitution on the oracle's blocks
    wr = np.zeros((nt, ne))
    for k in range(nt):
        rhs = br[k] - sum(Vr[k * (k + 1) // 2 + i] @ wr[i] for i in range(k))
        wr[k] = np.linalg.solve(Vr[k * (k + 1) // 2 + k], rhs)
    e4 = np.abs(w - wr).max() / np.abs(wr).max()
    # time marching: the inverses of all V^{k,k} (one batched Gauss-Jordan), then step by step
    wt, info_t = ctx.solve(torch.from_numpy(br).cuda(), method=HB_SOLVE_TIMEMARCH, tol=1e-8)
    wt = wt.cpu().numpy()
    e5 = np.abs(wt - wr).max() / np.abs(wr).max()
    ctx.close()
    say("  apply V %.2e, K %.2e; rhs %.2e; GMRES %d it, residual (oracle blocks) %.2e, "
        "solution %.2e; time marching: residual %.2e, solution %.2e"
        % (e1, e2, e3, info["iterations"], res, e4, info_t["rel_residual"], e5))
    assert e1 <= 1e-12 and e2 <= 1e-12 and e3 <= 1e-12
    assert info["converged"] and info["rel_residual"] <= 1e-8 and res <= 1.01e-8
    assert e4 <= 1e-6
    assert info_t["converged"] and info_t["rel_residual"] <= 1e-12 and e5 <= 1e-10


def test_nu_unsupported_entry_points(torch):
    from paper_2102_09811_amd import (HB_DTYPE_F32, HB_OP_D, HB_OP_K, HB_OP_V, HB_PREC_MIXED,
                                      HB_SOLVE_MIXED_IR, HBError, NonuniformContext)
    v, t = octahedron()
    with pytest.raises(HBError) as ei:  # nodes must start at 0 and increase
        NonuniformContext(v, t, 1.0, np.array([0.0, 0.5, 0.5, 1.0]))
    assert ei.value.code == -1
    with pytest.raises(HBError) as ei:
        NonuniformContext(v, t, 1.0, GRID, storage=HB_DTYPE_F32)
    assert ei.value.code == -1
    ctx = NonuniformContext(v, t, 1.0, GRID)
    for call in (lambda: ctx.assemble(HB_OP_V | HB_OP_D),
                 lambda: ctx.assemble(HB_OP_V, precision=HB_PREC_MIXED)):
        with pytest.raises(HBError) as ei:
            call()
        assert ei.value.code == -1
    ctx.assemble(HB_OP_V | HB_OP_K)
    b = torch.ones((ctx.n_t, ctx.n_tris), dtype=torch.float64, device="cuda")
    with pytest.raises(HBError) as ei:
        ctx.solve(b, method=HB_SOLVE_MIXED_IR)
    assert ei.value.code == -1
    ctx.close()


@pytest.mark.parametrize("case", ["octa_irregular9", "cube2_graded12"])
def test_nu_repr_matches_oracle(torch, case):
    """Potentials V~w and W g on the non-uniform grid against the oracle (long double closed
    forms) at points inside the mesh, at t = 0, at grid times, inside intervals and at t = T."""
    from paper_2102_09811_amd import NonuniformContext
    mesh, tn, alpha, _, _ = CASES[case]
    v, t = mesh()
    nt = len(tn) - 1
    rng = np.random.default_rng(17)
    w = rng.standard_normal((nt, len(t)))
    g = rng.standard_normal((nt, len(v)))
    c = v.mean(axis=0)
    times = [0.0, tn[1], 0.5 * (tn[2] + tn[3]), tn[nt // 2], 0.9 * tn[-1] + 0.1 * tn[-2], tn[-1]]
    pts = np.array([[c[0] + 0.1 * rng.standard_normal(), c[1] + 0.1 * rng.standard_normal(),
                     c[2] + 0.1 * rng.standard_normal(), s] for s in times for _ in range(3)])
    say("nonuniform potentials %s: %d points" % (case, len(pts)))
    sl_r, dl_r = oracle.repr_eval_nonuniform(v, t, alpha, tn, w, g, pts)
    ctx = NonuniformContext(v, t, alpha, tn)
    u, sl, dl = ctx.eval_repr(torch.from_numpy(pts).cuda(), torch.from_numpy(w).cuda(),
                              torch.from_numpy(g).cuda(), parts=True)
    ctx.close()
    sl, dl, u = sl.cpu().numpy(), dl.cpu().numpy(), u.cpu().numpy()
    es = np.abs(sl - sl_r).max() / np.abs(sl_r).max()
    ed = np.abs(dl - dl_r).max() / np.abs(dl_r).max()
    eu = np.abs(u - (sl_r - dl_r)).max() / np.abs(sl_r - dl_r).max()
    say("  single layer %.2e, double layer %.2e, u %.2e" % (es, ed, eu))
    assert es <= 1e-11 and ed <= 1e-11 and eu <= 1e-11
