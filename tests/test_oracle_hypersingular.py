"""Pins of the oracle's hypersingular operator (Sec. 3.3) and Neumann pipeline (Sec. 3.4, 6.1)
against mathematics the oracle does not use.

* D^{2,d}(r) against its definition as a double time integral of -alpha dG/dtau (mpmath, 2-D
  adaptive quadrature; dG/dtau written out from G), and D^{2,0} against alpha int_0^h G;
* the telescoping sum over d: sum_{d <= D} D^{2,d}(r) = alpha int_{Dh}^{(D+1)h} G(r, s) ds;
* surface curls of the p1 basis: a flat panel by hand, and their sum (the curl of 1) vanishes;
* D_h^1 annihilates spatially constant functions and is symmetric when V_h^d is;
* D_h^2 blocks are symmetric up to the regularised rules' error (exactly for separated pairs);
* end to end: the Neumann problem of Sec. 6.1 on the coarsest mesh (192 triangles, 8 steps)
  against the errors printed in Table 6.2;
* the p1 single layer V_h^{11} (the matrix of the paper's preconditioner for D_h) sums to the p0
  single layer over all entries (the p1 basis is a partition of unity).
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import downstream as ds
from synthetic import ExactSolution, box_points, cube, octahedron, space_time_points

mp.mp.dps = 30


def mp_G(rho, s, alpha):
    return (4 * mp.pi * alpha * s) ** mp.mpf(-1.5) * mp.e ** (-rho ** 2 / (4 * alpha * s))


def mp_dG_dtau(rho, t, tau, alpha):
    """d/dtau G(rho, t - tau) = -dG/ds at s = t - tau, from G = (4 pi alpha s)^{-3/2} e^{-rho^2/(4 alpha s)}."""
    s = t - tau
    return -mp_G(rho, s, alpha) * (rho ** 2 / (4 * alpha * s ** 2) - mp.mpf(3) / (2 * s))


@pytest.mark.parametrize("rho,d,alpha", [(0.3, 1, 0.5), (0.05, 2, 1.0), (0.8, 3, 0.5), (0.2, 6, 2.0)])
def test_D2_matches_defining_integral(rho, d, alpha):
    h = mp.mpf(1) / 8
    rho_m, al = mp.mpf(rho), mp.mpf(alpha)
    ref = -al * mp.quad(lambda t: mp.quad(lambda tau: mp_dG_dtau(rho_m, t, tau, al), [0, h]),
                        [d * h, (d + 1) * h])
    got = oracle.blockfun("D2", np.array([rho]), np.array([d]), float(h), alpha)[0]
    assert abs(got - float(ref)) <= 1e-13 * abs(float(ref))


@pytest.mark.parametrize("rho,alpha", [(0.3, 0.5), (0.05, 1.0), (1.2, 2.0)])
def test_D2_block0_is_time_integral_of_G(rho, alpha):
    h = mp.mpf(1) / 8
    ref = mp.mpf(alpha) * mp.quad(lambda t: mp_G(mp.mpf(rho), t, mp.mpf(alpha)), [0, h / 4, h])
    got = oracle.blockfun("D2", np.array([rho]), np.array([0]), float(h), alpha)[0]
    assert abs(got - float(ref)) <= 1e-13 * abs(float(ref))


def test_D2_telescoping_sum():
    h, alpha = 1.0 / 16, 0.7
    for rho in (0.01, 0.2, 0.9):
        for D in (0, 1, 5, 15, 40):
            d = np.arange(D + 1)
            s = oracle.blockfun("D2", np.full(D + 1, rho), d, h, alpha).astype(np.longdouble).sum()
            ref = alpha * mp.quad(lambda t: mp_G(mp.mpf(rho), t, mp.mpf(alpha)),
                                  [D * h, (D + 1) * h])
            assert abs(float(s) - float(ref)) <= 1e-13 * abs(float(ref)) + 1e-15 * float(np.abs(
                oracle.blockfun("D2", np.full(D + 1, rho), d, h, alpha)).max())


def test_surface_curls():
    v = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    t = np.array([[0, 1, 2]], dtype=np.int32)
    c = ds.surface_curls(v, t)[0]
    # lambda_0 = 1 - x - y, grad = (-1, -1, 0), curl = n x grad = (1, -1, 0); likewise the others
    assert np.allclose(c[0], [1, -1, 0]) and np.allclose(c[1], [0, 1, 0]) and np.allclose(c[2], [-1, 0, 0])
    vc, tc = cube(2)
    assert np.abs(ds.surface_curls(vc, tc).sum(axis=1)).max() < 1e-13


def test_D1_annihilates_constants_and_is_symmetric():
    v, t = octahedron()
    V, _ = oracle.assemble(v, t, 1.0, 1.0, 3)
    Vs = 0.5 * (V + V.transpose(0, 2, 1))
    D1 = ds.assemble_d1(Vs, v, t, 0.8)
    assert np.abs(D1 @ np.ones(len(v))).max() <= 1e-13 * np.abs(D1).max()
    assert np.abs(D1 - D1.transpose(0, 2, 1)).max() <= 1e-14 * np.abs(D1).max()


def test_D2_blocks_symmetric():
    v, t = cube(2)
    D2 = oracle.assemble_d2(v, t, 1.0, 1.0, 4)
    asym = np.abs(D2 - D2.transpose(0, 2, 1)).max() / np.abs(D2).max()
    assert 0 < asym < 1e-4
    # a pair of separated panels only: exactly symmetric
    vs = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [3.0, 0, 0], [4, 0, 0], [3, 1, 0]])
    ts = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    D2s = oracle.assemble_d2(vs, ts, 1.0, 1.0, 3)
    off = D2s[:, :3, 3:]
    assert np.abs(off - D2s[:, 3:, :3].transpose(0, 2, 1)).max() <= 1e-15 * np.abs(off).max()


def test_neumann_coarsest_level_table62():
    """Sec. 6.1, Neumann problem on 192 triangles x 8 steps, alpha = 0.5, u = G_alpha(x - y*, t):
    Table 6.2 prints L2 errors 3.14e-1 (u_h), 2.50e-1 (projection u*) and 5.16e-2 (potentials at
    10^4 points of [-0.5, 0.5]^3 x [0.25, 0.75]; 2000 seeded points here)."""
    alpha, T, nt = 0.5, 1.0, 8
    h = T / nt
    ex = ExactSolution(alpha, (0.0, 0.0, 1.5))
    v, t = cube(4, -1.0, 1.0)
    V, K = oracle.assemble(v, t, alpha, T, nt)
    D = ds.assemble_d1(V, v, t, alpha) + oracle.assemble_d2(v, t, alpha, T, nt)
    psi = ds.project_p0p0(v, t, nt, T, lambda x, n, tt: ex.flux(x, n, tt))
    u = ds.time_march(D, ds.rhs_neumann(K, ds.mass_p0p1(v, t), psi, h))
    e_u = ds.l2_error_p1p0(v, t, nt, T, u, ex.u)
    e_p = ds.l2_error_p1p0(v, t, nt, T, ds.project_p1p0(v, t, nt, T, ex.u), ex.u)
    pts = space_time_points(box_points(2000, -0.5, 0.5, seed=0), 0.25, 0.75, seed=0)
    sl, dl = oracle.repr_eval(v, t, alpha, T, nt, psi, u, pts)
    e_r = ds.relative_l2(ex.u(pts[:, :3], pts[:, 3]), sl - dl)
    assert abs(e_u / 3.14e-1 - 1) < 0.03
    assert abs(e_p / 2.50e-1 - 1) < 0.05
    assert abs(e_r / 5.16e-2 - 1) < 0.25


def test_V11_partition_of_unity_and_symmetry():
    """The p1 basis sums to one on every panel, so sum_{i,j} V11^d[i][j] = sum_{l,m} V^d[l][m]
    (V_h from the p0 assembly, a different code path), and V11 is symmetric up to the
    regularised rules' error."""
    v, t = octahedron()
    nt = 6
    V, _ = oracle.assemble(v, t, 0.8, 1.0, nt)
    V11 = oracle.assemble_v11(v, t, 0.8, 1.0, nt)
    s11 = V11.reshape(nt, -1).sum(1)
    s0 = V.reshape(nt, -1).sum(1)
    assert np.abs(s11 - s0).max() <= 1e-13 * np.abs(s0).max()
    asym = np.abs(V11 - V11.transpose(0, 2, 1)).max() / np.abs(V11).max()
    assert asym < 1e-4
