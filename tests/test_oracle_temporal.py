"""Pins of the oracle's temporal part against mathematics the oracle does not use.

* mpmath at 40 digits evaluates the paper's closed forms (Sec. 3.1, 3.2, summary Sec. 4) and,
  independently, the defining time integrals of V^d / K^d (hat-weighted integrals of the heat
  kernel, Sec. 3.1 eq. for V^d) by adaptive quadrature.
* limits printed in the paper (Sec. 3.1 / 3.2 "stable evaluations");
* derivative identities dG^{dtau dt}/ddelta = G^{dtau}, dG^{dtau}/ddelta = -G, and
  K^d / (r.n) = -(alpha/rho) dV^d/drho (the normal derivative passes through the time integrals);
* the telescoping sum over d of the block functions.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle

mp.mp.dps = 40


def mp_G(rho, s, alpha):
    return (4 * mp.pi * alpha * s) ** mp.mpf(-1.5) * mp.e ** (-rho ** 2 / (4 * alpha * s))


def mp_Gn_rn(rho, s, alpha):
    return mp.e ** (-rho ** 2 / (4 * alpha * s)) / (16 * (mp.pi * alpha) ** mp.mpf(1.5) * s ** mp.mpf(2.5))


def mp_closed(which, rho, delta, alpha):
    rho, delta, alpha = mp.mpf(rho), mp.mpf(delta), mp.mpf(alpha)
    z = rho / (2 * mp.sqrt(alpha * delta))
    if which == "g1":
        return mp.erf(z) / (4 * mp.pi * alpha * rho)
    if which == "F":
        return ((rho / (2 * alpha ** 2) + delta / (alpha * rho)) * mp.erf(z)
                + mp.sqrt(delta / (mp.pi * alpha ** 3)) * mp.e ** (-z * z)) / (4 * mp.pi)
    if which == "Fn_rn":
        return -((1 / (2 * alpha) - delta / rho ** 2) * mp.erf(z)
                 + mp.sqrt(delta) / (rho * mp.sqrt(mp.pi * alpha)) * mp.e ** (-z * z)) / (4 * mp.pi * rho)
    if which == "g1n_rn":
        return (mp.erf(z) / rho - mp.e ** (-z * z) / mp.sqrt(mp.pi * alpha * delta)) / (4 * mp.pi * rho ** 2)
    raise ValueError(which)


RHOS = [1e-4, 3e-3, 0.05, 0.3, 1.0, 2.5]
DELTAS = [1e-4, 1.0 / 64, 0.25, 1.0, 3.0]
ALPHAS = [0.1, 1.0, 10.0]


@pytest.mark.parametrize("which", ["g1", "F", "Fn_rn", "g1n_rn"])
@pytest.mark.parametrize("alpha", ALPHAS)
def test_closed_forms_match_mpmath(which, alpha):
    rho, delta = np.meshgrid(RHOS, DELTAS)
    got = oracle.temporal(which, rho, delta, alpha)
    worst = 0.0
    for r, d, g in zip(rho.ravel(), delta.ravel(), got):
        with mp.workdps(60):
            ref = mp_closed(which, r, d, alpha)
        worst = max(worst, float(abs((g - ref) / ref)))
    assert worst < 2e-15, worst


def test_limits_printed_in_paper():
    a = 0.7
    rho = np.array([0.2, 1.3])
    # delta -> 0+
    assert np.allclose(oracle.temporal("F", rho, 1e-300, a), rho / (8 * np.pi * a * a), rtol=1e-15)
    assert np.allclose(oracle.temporal("F", rho, 0.0, a), rho / (8 * np.pi * a * a), rtol=1e-15)
    assert np.allclose(oracle.temporal("g1", rho, 1e-300, a), 1 / (4 * np.pi * a * rho), rtol=1e-15)
    assert np.allclose(oracle.temporal("Fn_rn", rho, 1e-300, a), -1 / (8 * np.pi * a * rho), rtol=1e-15)
    assert np.allclose(oracle.temporal("g1n_rn", rho, 1e-300, a), 1 / (4 * np.pi * rho ** 3), rtol=1e-15)
    # rho -> 0+
    delta = np.array([0.01, 0.5])
    lim = np.sqrt(delta) / (2 * np.sqrt(np.pi ** 3 * a ** 3))
    assert np.allclose(oracle.temporal("F", 1e-12, delta, a), lim, rtol=1e-10)
    assert np.allclose(oracle.temporal("F", 0.0, delta, a), lim, rtol=1e-15)
    # alpha dG^{dtau dt}/dn -> 0 as rho -> 0 (here divided by r.n, it stays bounded)
    assert np.all(np.abs(oracle.temporal("Fn_rn", 1e-9, delta, a) * 1e-9) < 1e-8)


def test_derivative_identities():
    a = 0.9
    rho = np.array([0.05, 0.4, 1.1])
    for delta in (0.03, 0.5):
        eps = 1e-6 * delta
        dF = (oracle.temporal("F", rho, delta + eps, a) - oracle.temporal("F", rho, delta - eps, a)) / (2 * eps)
        assert np.allclose(dF, oracle.temporal("g1", rho, delta, a), rtol=1e-8)
        dg = (oracle.temporal("g1", rho, delta + eps, a) - oracle.temporal("g1", rho, delta - eps, a)) / (2 * eps)
        G = (4 * np.pi * a * delta) ** -1.5 * np.exp(-rho ** 2 / (4 * a * delta))
        assert np.allclose(dg, -G, rtol=1e-7)
        # d/ddelta of alpha dG^{dtau dt}/dn = alpha dG^{dtau}/dn
        dFn = (oracle.temporal("Fn_rn", rho, delta + eps, a) - oracle.temporal("Fn_rn", rho, delta - eps, a)) / (2 * eps)
        assert np.allclose(dFn, oracle.temporal("g1n_rn", rho, delta, a), rtol=1e-7)


def _mp_block(which, rho, d, h, alpha):
    """Exact V^d(r) / (K^d(r)/r.n) from the defining time integral, by mpmath quadrature."""
    rho, h, alpha = mp.mpf(rho), mp.mpf(h), mp.mpf(alpha)
    f = mp_G if which == "V" else mp_Gn_rn
    if d == 0:
        return mp.quad(lambda s: (h - s) * f(rho, s, alpha), [0, h / 4, h])
    return mp.quad(lambda s: (h - abs(s - d * h)) * f(rho, s, alpha),
                   [(d - 1) * h, (d - 1) * h + h / 4, d * h, (d + 1) * h])


@pytest.mark.parametrize("which", ["V", "K"])
@pytest.mark.parametrize("tmode", [0, 1, 2])
def test_block_functions_match_time_integral(which, tmode):
    """Errors are measured against the size a block entry of this d can reach (the value at a
    near distance), because far entries are exponentially small differences of O(1) terms."""
    h, alpha = 1.0 / 64, 1.0
    ds = [0, 1, 2, 3, 7, 8, 15, 16, 17, 40, 63]
    rhos = np.array([2e-3, 0.05, 0.2, 0.8, 1.9])
    worst = 0.0
    for d in ds:
        got = oracle.blockfun(which, rhos, np.full(len(rhos), d), h, alpha, tmode)
        refs = [_mp_block(which, r, d, h, alpha) for r in rhos]
        # K^d / (r.n) is multiplied by r.n <= rho in a block entry
        wts = rhos if which == "K" else np.ones_like(rhos)
        scale = max(abs(float(r)) * w for r, w in zip(refs[1:], wts[1:]))
        for r, g, w in zip(refs, got, wts):
            worst = max(worst, float(abs(g - r)) * w / scale)
    tol = 1e-13 if tmode != 1 else 1e-12   # closed form at d = 63 loses ~4 d^2 ulp (long double)
    assert worst < tol, worst


def test_K_is_normal_derivative_of_V():
    """K^d(r) = alpha dV^d/dn_y = -alpha (dV^d/drho) (r.n)/rho  (Sec. 3.2)."""
    h, a = 1.0 / 16, 1.3
    rho = np.array([0.07, 0.3, 0.9])
    for d in (0, 1, 2, 5, 20):
        eps = 1e-5 * rho
        dV = (oracle.blockfun("V", rho + eps, d, h, a) - oracle.blockfun("V", rho - eps, d, h, a)) / (2 * eps)
        assert np.allclose(oracle.blockfun("K", rho, d, h, a), -a * dV / rho, rtol=2e-7), d


def test_telescoping_sum():
    """sum_{d=0}^{D} V^d = h G^{dtau}(r, 0) - [G^{dtau dt}((D+1)h) - G^{dtau dt}(Dh)] and the same
    for K (the block integrals tile the time axis)."""
    h, a = 1.0 / 32, 0.5
    rho = np.array([0.01, 0.2, 1.0])
    D = 40
    sV = sum(oracle.blockfun("V", rho, d, h, a) for d in range(D + 1))
    sK = sum(oracle.blockfun("K", rho, d, h, a) for d in range(D + 1))
    refV = h / (4 * np.pi * a * rho) - (oracle.temporal("F", rho, (D + 1) * h, a) - oracle.temporal("F", rho, D * h, a))
    refK = h / (4 * np.pi * rho ** 3) - (oracle.temporal("Fn_rn", rho, (D + 1) * h, a) - oracle.temporal("Fn_rn", rho, D * h, a))
    assert np.allclose(sV, refV, rtol=1e-13)
    assert np.allclose(sK, refK, rtol=1e-13)
