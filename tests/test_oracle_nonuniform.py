"""Pins of the oracle's blocks on non-uniform time grids (the paper's outlook, Sec. 7, with the
block integrals of Sec. 3.1 and 3.2 at general interval endpoints).

* the defining double time integral of G_alpha (and of alpha dG/dn / (r . n)) over test interval
  I_k and trial interval I_i, by mpmath at 30 digits (2-D over the rectangle for i < k, the
  triangle tau < t as the 1-D form for i = k) -- independent of the four-term difference and of
  the trapezoid quadrature the oracle uses;
* additivity: splitting a trial interval into two splits its blocks into the sum of two blocks,
  splitting a test interval likewise (on the diagonal the later half against the earlier one
  adds a third block) -- exact identities that any wrong index, sign or endpoint breaks;
* causality sum: sum over i <= k of V^{k,i}(r) = h_k G^{dtau}(r, 0) - [F(t_{k+1}) - F(t_k)];
* a uniform grid reproduces the Toeplitz blocks V^{k-i}, K^{k-i} of the uniform assembly (a
  different formula: second differences and the hat quadrature);
* on a mesh, the same two identities hold for the assembled blocks.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from synthetic import cube, octahedron

GRID = np.array([0.0, 0.05, 0.12, 0.2, 0.33, 0.45, 0.6, 0.72, 0.9, 1.0])  # graded, 9 intervals


def G_exact(rho, s, alpha, which):
    """G_alpha(rho, s) (which 'V') or alpha dG/dn_y / (r . n_y) (which 'K'), s > 0."""
    if s <= 0:
        return mp.mpf(0)
    e = mp.exp(-rho ** 2 / (4 * alpha * s))
    if which == "V":
        return e / (4 * mp.pi * alpha * s) ** mp.mpf(1.5)
    return e / (16 * (mp.pi * alpha) ** mp.mpf(1.5) * s ** mp.mpf(2.5))


def block_exact(rho, k, i, t, alpha, which):
    mp.mp.dps = 30
    rho, alpha = mp.mpf(rho), mp.mpf(alpha)
    tk, tk1, ti, ti1 = (mp.mpf(float(x)) for x in (t[k], t[k + 1], t[i], t[i + 1]))
    f = lambda s: G_exact(rho, s, alpha, which)  # noqa: E731
    if i == k:   # int_{I_k} int_{t_k}^{t} G(t - tau) dtau dt = int_0^{h} (h - s) G(s) ds
        h = tk1 - tk
        return mp.quad(lambda s: (h - s) * f(s), [0, h / 64, h / 8, h])
    return mp.quad(lambda tt, tau: f(tt - tau), [tk, tk1], [ti, ti1])


@pytest.mark.parametrize("which", ["V", "K"])
def test_blocks_against_defining_integral(which):
    t = GRID
    alpha = 0.7
    cases = [(0.03, 0, 0), (0.4, 3, 3), (0.2, 4, 3), (0.05, 4, 3), (0.3, 8, 0), (0.6, 8, 5),
             (0.01, 6, 2), (1.2, 7, 1)]
    for rho, k, i in cases:
        ref = float(block_exact(rho, k, i, t, alpha, which))
        got = oracle.nu_blockfun(which, rho, k, i, t, alpha)[0]
        assert abs(got - ref) <= 1e-13 * abs(ref), (which, rho, k, i, got, ref)


def test_additivity_and_causality_sum():
    t = GRID
    alpha = 1.3
    rho = np.array([1e-3, 0.02, 0.1, 0.35, 0.9, 2.0])
    nt = len(t) - 1
    for j in (0, 3, 7):
        t2 = np.sort(np.append(t, 0.5 * (t[j] + t[j + 1])))     # interval j split in two: j, j + 1
        for which in ("V", "K"):
            f = lambda k, i, g: oracle.nu_blockfun(which, rho, k, i, g, alpha)  # noqa: E731
            for k in range(nt):
                for i in range(k + 1):
                    A = f(k, i, t)
                    k2 = k if k < j else k + 1                                  # index on t2
                    i2 = i if i < j else i + 1
                    if i == j and k == j:
                        B = f(j, j, t2) + f(j + 1, j, t2) + f(j + 1, j + 1, t2)
                    elif i == j:
                        B = f(k2, j, t2) + f(k2, j + 1, t2)
                    elif k == j:
                        B = f(j, i2, t2) + f(j + 1, i2, t2)
                    else:
                        B = f(k2, i2, t2)
                    assert np.allclose(A, B, rtol=1e-13, atol=0), (which, j, k, i, A, B)
    # sum over the trial intervals: h_k G^{dtau}(rho, 0) - [F(t_{k+1}) - F(t_k)] (the reference's
    # three terms are rounded to double before they cancel: compared on their scale)
    for k in range(nt):
        tot = sum(oracle.nu_blockfun("V", rho, k, i, t, alpha) for i in range(k + 1))
        terms = ((t[k + 1] - t[k]) * oracle.temporal("g1", rho, 0.0, alpha),
                 oracle.temporal("F", rho, t[k + 1], alpha), oracle.temporal("F", rho, t[k], alpha))
        ref = terms[0] - terms[1] + terms[2]
        scale = np.max(np.abs(terms), axis=0)
        assert np.all(np.abs(tot - ref) <= 1e-14 * scale), (k, tot, ref)


def test_uniform_grid_gives_toeplitz_blocks():
    v, t = cube(2)
    nt, T, alpha = 10, 1.0, 0.8
    V, K = oracle.assemble_nonuniform(v, t, alpha, np.arange(nt + 1) * T / nt)
    Vu, Ku = oracle.assemble(v, t, alpha, T, nt)
    for k in range(nt):
        for i in range(k + 1):
            e = k * (k + 1) // 2 + i
            assert np.abs(V[e] - Vu[k - i]).max() <= 1e-13 * np.abs(Vu[k - i]).max(), (k, i)
            assert np.abs(K[e] - Ku[k - i]).max() <= 1e-13 * np.abs(Ku[k - i]).max(), (k, i)


def test_assembled_blocks_split_interval():
    """Splitting trial/test interval j of the grid: the assembled blocks add up (octahedron, every
    pair class)."""
    v, t = octahedron()
    g = np.array([0.0, 0.1, 0.25, 0.5, 0.6, 1.0])
    j = 2
    g2 = np.sort(np.append(g, 0.5 * (g[j] + g[j + 1])))
    V, K = oracle.assemble_nonuniform(v, t, 0.9, g)
    V2, K2 = oracle.assemble_nonuniform(v, t, 0.9, g2)
    e = lambda k, i: k * (k + 1) // 2 + i  # noqa: E731
    for A, A2 in ((V, V2), (K, K2)):
        for k in range(len(g) - 1):
            k2 = k if k < j else k + 1
            sc = np.abs(A[e(k, 0)]).max()
            if k == j:
                B = A2[e(j, 0)] + A2[e(j + 1, 0)]
                assert np.abs(A[e(k, 0)] - B).max() <= 1e-13 * sc
            if k >= j:
                if k == j:
                    B = A2[e(j, j)] + A2[e(j + 1, j)] + A2[e(j + 1, j + 1)]
                else:
                    B = A2[e(k2, j)] + A2[e(k2, j + 1)]
                assert np.abs(A[e(k, j)] - B).max() <= 1e-13 * np.abs(A[e(k, j)]).max(), k


def _repr_inputs(nt, seed):
    v, t = octahedron()
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nt, len(t)))
    u = rng.standard_normal((nt, len(v)))
    return v, t, w, u


def test_repr_uniform_grid_matches_uniform_oracle():
    """The non-uniform representation formula on the uniform grid t_j = j T / nt equals the
    uniform oracle's (points in the current interval, at grid times, at t = 0 and t = T)."""
    nt, T, alpha = 7, 1.3, 0.8
    v, t, w, u = _repr_inputs(nt, 41)
    ts = [0.0, 0.05, T / nt, 2.5 * T / nt, 0.999, T]
    pts = np.array([[0.1, -0.05, 0.12, s] for s in ts] + [[-0.2, 0.1, 0.0, 0.77]])
    sl0, dl0 = oracle.repr_eval(v, t, alpha, T, nt, w, u, pts)
    sl1, dl1 = oracle.repr_eval_nonuniform(v, t, alpha, np.arange(nt + 1) * (T / nt), w, u, pts)
    assert np.abs(sl1 - sl0).max() <= 1e-14 * np.abs(sl0).max()
    assert np.abs(dl1 - dl0).max() <= 1e-14 * np.abs(dl0).max()


@pytest.mark.parametrize("coarse", ["uniform", "graded"])
def test_repr_refined_grid_with_repeated_data(coarse):
    """Splitting every interval at an interior point and repeating its data on both halves leaves
    the potentials unchanged (additivity of the time integrals); from a uniform coarse grid this
    ties the non-uniform formula to the uniform oracle."""
    alpha = 0.6
    tn = np.linspace(0.0, 1.0, 6) if coarse == "uniform" else GRID
    nt = len(tn) - 1
    v, t, w, u = _repr_inputs(nt, 43)
    rng = np.random.default_rng(44)
    cut = tn[:-1] + (0.2 + 0.6 * rng.random(nt)) * np.diff(tn)
    fine = np.sort(np.concatenate([tn, cut]))
    rep = np.repeat(np.arange(nt), 2)
    pts = np.array([[0.05, 0.1, -0.1, s] for s in (0.03, tn[2], 0.5 * (tn[3] + cut[3]), 0.97, 1.0)])
    if coarse == "uniform":
        slc, dlc = oracle.repr_eval(v, t, alpha, 1.0, nt, w, u, pts)
    else:
        slc, dlc = oracle.repr_eval_nonuniform(v, t, alpha, tn, w, u, pts)
    slf, dlf = oracle.repr_eval_nonuniform(v, t, alpha, fine, w[rep], u[rep], pts)
    assert np.abs(slf - slc).max() <= 1e-13 * np.abs(slc).max()
    assert np.abs(dlf - dlc).max() <= 1e-13 * np.abs(dlc).max()
