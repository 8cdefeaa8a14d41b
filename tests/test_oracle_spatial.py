"""Pins of the oracle's spatial quadrature (Sec. 3.1 "Galerkin weights", Sec. 5.2).

* Radon's 7-point rule integrates every monomial of degree <= 5 exactly (and not degree 6).
* The regularised [0,1]^4 rules integrate polynomials on T x T exactly (the maps tile T x T).
* Singular integrals over the unit square, split into touching triangles, converge to closed
  values: int int |x-y|^{-1} and int int |x-y| over the square reduce to 1D integrals over the
  difference vector (evaluated here by mpmath, not by the oracle's rules).
* The Laplace double layer (the d -> infinity sum of the heat double-layer blocks divided by h)
  integrates to -1/2 per unit area on a closed surface (solid angle), which fixes the normal's
  orientation and the sign of r = x - y.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from synthetic import cube, icosphere, octahedron, tetrahedron


def tri_monomial(a, b):
    """int over T = {0 <= x2 <= x1 <= 1} of x1^a x2^b."""
    return 1.0 / ((b + 1) * (a + b + 2))


def test_radon7_exact_to_degree5():
    lam, w = oracle.triangle_rule(0, 7)
    assert abs(w.sum() - 1) < 1e-15
    # reference point x1 = lam1 + lam2, x2 = lam2 on T (|T| = 1/2)
    x1, x2 = lam[:, 1] + lam[:, 2], lam[:, 2]
    for deg in range(7):
        errs = []
        for a in range(deg + 1):
            b = deg - a
            q = 0.5 * np.sum(w * x1 ** a * x2 ** b)
            errs.append(abs(q - tri_monomial(a, b)) / tri_monomial(a, b))
        if deg <= 5:
            assert max(errs) < 1e-14, (deg, errs)
        else:
            assert max(errs) > 1e-6


def test_gauss_legendre_exactness():
    for n in (1, 2, 4, 7, 12):
        x, w = oracle.gauss_legendre01(n)
        for k in range(2 * n):
            assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15
        if n <= 4:
            assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-10


def test_collapsed_triangle_rule():
    lam, w = oracle.triangle_rule(1, 8)
    x1, x2 = lam[:, 1] + lam[:, 2], lam[:, 2]
    for a, b in [(0, 0), (3, 4), (7, 2), (1, 6)]:
        assert abs(0.5 * np.sum(w * x1 ** a * x2 ** b) - tri_monomial(a, b)) < 1e-15


@pytest.mark.parametrize("cls", [1, 2, 3])
def test_regularised_rules_tile_TxT(cls):
    xh, yh, w = oracle.ss_rule(cls, 6)
    assert abs(w.sum() - 0.25) < 1e-15
    rng = np.random.default_rng(cls)
    for _ in range(12):
        a, b, c, d = rng.integers(0, 3, size=4)
        q = np.sum(w * xh[:, 0] ** a * xh[:, 1] ** b * yh[:, 0] ** c * yh[:, 1] ** d)
        ex = tri_monomial(a, b) * tri_monomial(c, d)
        assert abs(q - ex) / ex < 1e-13


def test_pair_classification_and_weights():
    v, t = octahedron()
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)
    counts = {0: 0, 1: 0, 2: 0, 3: 0}
    for a in range(len(t)):
        for b in range(len(t)):
            p = oracle.pair_points(v, t, a, b, 4)
            counts[p["cls"]] += 1
            assert abs(p["W"].sum() - area[a] * area[b]) < 1e-14
            assert np.allclose(p["phi"].sum(1), 1.0)
            # phi are the barycentric coordinates of y in the trial panel's original order
            assert np.allclose(p["phi"] @ v[t[b]], p["y"], atol=1e-14)
            # test points lie on the test panel (plane), trial points on the trial panel
            n = np.cross(v[t[a, 1]] - v[t[a, 0]], v[t[a, 2]] - v[t[a, 0]])
            assert np.allclose((p["x"] - v[t[a, 0]]) @ n, 0, atol=1e-14)
    # octahedron: 8 identical, 24 ordered edge pairs, 24 vertex pairs, 8 antipodal separated
    assert counts == {3: 8, 2: 24, 1: 24, 0: 8}
    v, t = tetrahedron()
    cls = {oracle.pair_points(v, t, a, b, 2)["cls"] for a in range(4) for b in range(4) if a != b}
    assert cls == {2}


def _square_reference(power):
    """int_{[0,1]^2} int_{[0,1]^2} |x - y|^power = 4 int_{[0,1]^2} (1-u1)(1-u2) |u|^power du,
    in polar coordinates with the radial integral done exactly."""
    mp.mp.dps = 30

    def inner(th):
        c, s = mp.cos(th), mp.sin(th)
        R = 1 / max(c, s)
        p = power + 1  # r^power * r dr
        return R ** (p + 1) / (p + 1) - (c + s) * R ** (p + 2) / (p + 2) + c * s * R ** (p + 3) / (p + 3)
    return float(4 * mp.quad(inner, [0, mp.pi / 4, mp.pi / 2]))


def _square_meshes():
    v2 = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=float)
    t2 = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    v4 = np.vstack([v2, [[0.5, 0.5, 0]]])
    t4 = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], dtype=np.int32)
    return [(v2, t2), (v4, t4)]


@pytest.mark.parametrize("power", [-1, 1])
def test_singular_square_integrals_converge(power):
    ref = _square_reference(power)
    if power == -1:   # classical value 4 ln(1 + sqrt 2) - (4/3)(sqrt 2 - 1)
        assert abs(ref - (4 * math.log(1 + math.sqrt(2)) - 4.0 / 3.0 * (math.sqrt(2) - 1))) < 1e-14
    else:             # mean distance in the unit square (2 + sqrt 2 + 5 ln(1 + sqrt 2)) / 15
        assert abs(ref - (2 + math.sqrt(2) + 5 * math.log(1 + math.sqrt(2))) / 15) < 1e-14
    for v, t in _square_meshes():
        errs = []
        for M in (2, 4, 8, 12):
            tot = 0.0
            for a in range(len(t)):
                for b in range(len(t)):
                    p = oracle.pair_points(v, t, a, b, M)
                    rho = np.linalg.norm(p["x"] - p["y"], axis=1)
                    tot += np.sum(p["W"] * rho ** power)
            errs.append(abs(tot - ref) / ref)
        # geometric convergence in the Gauss order of the regularised rule
        assert errs[1] < 3e-4 and errs[2] < 3e-7 and errs[3] < 3e-10, errs
        assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("mesh", ["cube", "icosphere"])
def test_double_layer_solid_angle(mesh):
    v, t = cube(3) if mesh == "cube" else icosphere(1)
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    for a in (0, len(t) // 2):
        tot = 0.0
        for b in range(len(t)):
            p = oracle.pair_points(v, t, a, b, 6)
            r = p["x"] - p["y"]
            rho = np.linalg.norm(r, axis=1)
            tot += np.sum(p["W"] * (r @ nrm[b]) / (4 * np.pi * rho ** 3))
        # -1/2 per unit test area, up to the 7-point rule's error on near, separated pairs
        assert abs(tot / area[a] + 0.5) < 2e-3, tot / area[a]
