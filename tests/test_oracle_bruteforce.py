"""Pin of the oracle's separated-pair entries against a brute-force evaluation in space and time.

For two small, well separated panels the entries V_h^d[l][m] and the trial-vertex parts of
K_h^d[l][.] (Sec. 3.1, 3.2) are computed here from their definitions alone: high-order Gauss on
both triangles (collapsed Gauss-Legendre) and Gauss-Legendre in time over the two halves of the
hat function of block d, with the heat kernel G_alpha and its normal derivative
alpha dG/dn_y = (r . n_y) / (2 s) G (r = x - y) written out here.  The oracle uses Radon's 7-point
rule on both panels (degree 5), so it must agree within that rule's error, and the difference must
shrink like size^6 when both panels are halved.
"""
import numpy as np

import oracle

ALPHA, T, NT = 1.0, 1.0, 6
H = T / NT


def tri_rule(n):
    """Collapsed Gauss-Legendre on the reference triangle: barycentric (n^2, 3), weights sum 1."""
    g, w = np.polynomial.legendre.leggauss(n)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    u, v = np.meshgrid(g, g, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    s, t = u.ravel(), (v * (1.0 - u)).ravel()          # (s, t) in the triangle s + t <= 1
    W = 2.0 * (wu * wv * (1.0 - u)).ravel()           # area of the reference triangle is 1/2
    lam = np.stack([1.0 - s - t, s, t], axis=1)
    return lam, W


def heat_kernel(rho, s):
    return (4.0 * np.pi * ALPHA * s) ** -1.5 * np.exp(-rho ** 2 / (4.0 * ALPHA * s))


def time_nodes(d, n=40):
    """Nodes and weights of int (h - |s - d h|)_+ f(s) ds over s > 0 (the block-d hat function),
    Gauss-Legendre on each linear piece."""
    g, w = np.polynomial.legendre.leggauss(n)
    ss, ww = [], []
    for a, b in ((max(0, d - 1) * H, d * H), (d * H, (d + 1) * H)):
        if b <= a:
            continue
        s = 0.5 * (b - a) * (g + 1.0) + a
        ss.append(s)
        ww.append(0.5 * (b - a) * w * (H - np.abs(s - d * H)))
    return np.concatenate(ss), np.concatenate(ww)


def brute_blocks(verts, tris, l, m, n_space=10):
    lam, W = tri_rule(n_space)
    P, Q = verts[tris[l]], verts[tris[m]]
    x, y = lam @ P, lam @ Q
    area = lambda X: 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))  # noqa: E731
    nm = np.cross(Q[1] - Q[0], Q[2] - Q[0])
    nm /= np.linalg.norm(nm)
    r = x[:, None, :] - y[None, :, :]
    rho = np.linalg.norm(r, axis=2)
    rn = r @ nm
    w2 = np.outer(W, W) * area(P) * area(Q)
    V = np.empty(NT)
    K = np.empty((NT, 3))
    for d in range(NT):
        s, ws = time_nodes(d)
        g = heat_kernel(rho[..., None], s) @ ws                          # int hat * G
        gn = (heat_kernel(rho[..., None], s) / (2.0 * s)) @ ws            # int hat * G / (2 s)
        V[d] = np.sum(w2 * g)
        for k in range(3):
            K[d, k] = np.sum(w2 * rn * gn * lam[None, :, k])
    return V, K


def pair(scale):
    """Two parallel triangles of size ~ scale facing each other at distance 0.5."""
    base = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    top = np.array([[0.2, 0.1, 0.0], [0.1, 1.1, 0.0], [1.0, 0.3, 0.0]])
    verts = np.vstack([scale * base, scale * top + [0.0, 0.0, 0.5]])
    return verts, np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)


def test_separated_entries_against_brute_force():
    errs = []
    for scale in (0.4, 0.2, 0.1):
        verts, tris = pair(scale)
        Vb, Kb = brute_blocks(verts, tris, 0, 1)
        Vo, Ko = oracle.pair_blocks(verts, tris, ALPHA, T, NT, 0, 1)
        # the brute force itself is converged: a finer spatial rule changes nothing
        Vb2, Kb2 = brute_blocks(verts, tris, 0, 1, n_space=14)
        assert np.abs(Vb2 - Vb).max() <= 1e-12 * np.abs(Vb).max()
        assert np.abs(Kb2 - Kb).max() <= 1e-12 * np.abs(Kb).max()
        eV = np.abs(Vo - Vb).max() / np.abs(Vb).max()
        eK = np.abs(Ko - Kb).max() / np.abs(Kb).max()
        errs.append((eV, eK))
    (v0, k0), (v1, k1), (v2, k2) = errs
    # the 7-point rule is exact to degree 5: errors of order size^6, a factor approaching 64 per
    # halving (measured 28 then 53 for V, 20 then 38 for K); a wrong weight, area, normal or basis
    # value would leave an O(1) error, a wrong node a factor of about 4
    assert v0 < 1e-3 and k0 < 1e-3, errs
    assert v2 < 1e-6 and k2 < 1e-5, errs
    assert v0 / v1 > 15 and k0 / k1 > 15, errs
    assert v1 / v2 > 30 and k1 / k2 > 30, errs


def test_touching_entries_against_brute_force():
    """Identical, edge- and vertex-sharing panels of the octahedron.  From block d = 2 on the time
    integral stays away from s = 0, the integrand is smooth on the pair and the brute force above
    converges; the oracle's regularised (Sauter-Schwab type) rules must approach it quickly as
    their order grows (Gauss order 4, the production order, then 6 and 8).  Blocks 0 and 1 are
    singular: there the rules must converge among themselves.  K of an identical (flat) pair
    vanishes."""
    from synthetic import octahedron
    v, t = octahedron()
    share = [len(set(t[0]) & set(t[m])) for m in range(len(t))]
    Kscale = None
    for name, m in (("edge", share.index(2)), ("vertex", share.index(1)), ("identical", 0)):
        Vb, Kb = brute_blocks(v, t, 0, m, n_space=16)
        Vb2, Kb2 = brute_blocks(v, t, 0, m, n_space=20)
        assert np.abs(Vb2[2:] - Vb[2:]).max() <= 1e-13 * np.abs(Vb[2:]).max()
        res = {so: oracle.pair_blocks(v, t, ALPHA, T, NT, 0, m, ss_order=so) for so in (4, 6, 8)}
        eV = {so: np.abs(res[so][0][2:] - Vb2[2:]).max() / np.abs(Vb2[2:]).max() for so in res}
        assert eV[4] < 1e-4 and eV[8] < 1e-9 and eV[4] / eV[8] > 1e3, (name, eV)
        if name == "identical":
            assert np.abs(res[4][1]).max() <= 1e-12 * Kscale
        else:
            Kscale = np.abs(Kb2).max() if Kscale is None else max(Kscale, np.abs(Kb2).max())
            eK = {so: np.abs(res[so][1][2:] - Kb2[2:]).max() / np.abs(Kb2[2:]).max() for so in res}
            assert eK[4] < 1e-3 and eK[8] < 1e-8 and eK[4] / eK[8] > 1e3, (name, eK)
        # singular blocks 0, 1: the rules converge among themselves
        V4, V6, V8 = (res[so][0][:2] for so in (4, 6, 8))
        d46, d68 = np.abs(V4 - V8).max(), np.abs(V6 - V8).max()
        assert d68 <= 1e-5 * np.abs(V8).max() and d68 < d46 / 5, (name, d46, d68)


def p1p1_brute(v, t, kind, n_space=14):
    """All N_x x N_x blocks d >= 2 of V_h^{11} ('V11': the p1 x p1 single layer) or D_h^2 ('D2',
    Sec. 3.3: n_x . n_y times the time derivative part alpha int_{dh}^{(d+1)h} G(t) - G(t - h) dt)
    by brute force over every panel pair (smooth from d = 2 on)."""
    lam, W = tri_rule(n_space)
    g, gw = np.polynomial.legendre.leggauss(40)
    out = np.zeros((NT, len(v), len(v)))
    geo = []
    for tri in t:
        P = v[tri]
        c = np.cross(P[1] - P[0], P[2] - P[0])
        geo.append((lam @ P, 0.5 * np.linalg.norm(c), c / np.linalg.norm(c)))
    for l in range(len(t)):
        x, al, nl = geo[l]
        for m in range(len(t)):
            y, am, nm = geo[m]
            rho = np.linalg.norm(x[:, None, :] - y[None, :, :], axis=2)[..., None]
            w2 = np.outer(W, W) * al * am * (nl @ nm if kind == "D2" else 1.0)
            for d in range(2, NT):
                if kind == "V11":
                    s, ws = time_nodes(d)
                    kv = heat_kernel(rho, s) @ ws
                else:
                    a, b = d * H, (d + 1) * H
                    s, ws = 0.5 * (b - a) * (g + 1.0) + a, 0.5 * (b - a) * gw
                    kv = ALPHA * ((heat_kernel(rho, s) - heat_kernel(rho, s - H)) @ ws)
                out[d][np.ix_(t[l], t[m])] += lam.T @ (w2 * kv) @ lam
    return out


def test_p1p1_blocks_against_brute_force():
    """V_h^{11} and D_h^2 of the octahedron, blocks d >= 2, against brute force: the oracle's
    7-point (separated) and regularised (touching) rules agree within their error, which falls
    as the mesh shrinks relative to the kernel's width (measured 5e-4, 4e-5, 3e-6 at radius 1,
    0.5, 0.25); a wrong basis value, normal product or area would leave an O(1) error."""
    from synthetic import octahedron
    errs = {}
    for rad in (0.5, 0.25):
        v, t = octahedron(rad)
        for kind, fn in (("V11", oracle.assemble_v11), ("D2", oracle.assemble_d2)):
            ref = p1p1_brute(v, t, kind)
            got = fn(v, t, ALPHA, T, NT)
            errs[(rad, kind)] = max(np.abs(got[d] - ref[d]).max() / np.abs(ref[d]).max()
                                    for d in range(2, NT))
    for kind in ("V11", "D2"):
        e1, e2 = errs[(0.5, kind)], errs[(0.25, kind)]
        assert e1 < 1e-4 and e2 < 1e-5 and e1 / e2 > 8, errs


def potentials_brute(v, t, w, u, pt, n_space=16):
    """Single- and double-layer potentials (Sec. 3.5) at one point (x, t) off the surface for
    piecewise constant-in-time densities: w (p0 in space) and u (p1 in space), by Gauss on every
    panel and Gauss-Legendre in s = t - tau over each interval (the current one graded towards
    s = 0, where G is smooth but steep)."""
    lam, W = tri_rule(n_space)
    g, gw = np.polynomial.legendre.leggauss(60)
    seg = lambda a, b: (0.5 * (b - a) * (g + 1.0) + a, 0.5 * (b - a) * gw)  # noqa: E731
    x, tt = pt[:3], pt[3]
    sl = dl = 0.0
    for i in range(NT):
        a, b = i * H, min((i + 1) * H, tt)
        if b <= a:
            continue
        lo, hi = tt - b, tt - a
        pieces = [(lo, hi)] if lo > 0 else [(0.0, hi / 64), (hi / 64, hi / 8), (hi / 8, hi / 2),
                                            (hi / 2, hi)]
        s = np.concatenate([seg(*pc)[0] for pc in pieces])
        ws = np.concatenate([seg(*pc)[1] for pc in pieces])
        for l in range(len(t)):
            Q = v[t[l]]
            c = np.cross(Q[1] - Q[0], Q[2] - Q[0])
            area, n = 0.5 * np.linalg.norm(c), c / np.linalg.norm(c)
            r = x[None, :] - lam @ Q
            G = heat_kernel(np.linalg.norm(r, axis=1)[:, None], s[None, :])
            sl += w[i, l] * area * (W @ (G @ ws))
            dl += area * np.sum(W * ((G / (2.0 * s[None, :])) @ ws) * (r @ n) * (lam @ u[i, t[l]]))
    return sl, dl


def test_potentials_against_brute_force():
    """The oracle's potentials (closed-form time integrals) at points inside the octahedron, with
    its collapsed Gauss rule in space, against the brute force above: they converge together as
    the spatial order grows (order 16: below 1e-8 relative)."""
    from synthetic import octahedron
    v, t = octahedron()
    rng = np.random.default_rng(5)
    w = rng.standard_normal((NT, len(t)))
    u = rng.standard_normal((NT, len(v)))
    pts = np.array([[0.1, -0.05, 0.2, 0.37], [-0.2, 0.1, 0.0, 0.9], [0.05, 0.05, -0.1, 0.5],
                    [0.0, 0.2, 0.1, 1.0], [0.15, 0.0, 0.0, 0.1]])
    ref = np.array([potentials_brute(v, t, w, u, p) for p in pts])
    err = {}
    for order in (8, 16):
        sl, dl = oracle.repr_eval(v, t, ALPHA, T, NT, w, u, pts, rule_kind=1, rule_order=order)
        err[order] = (np.abs(sl - ref[:, 0]).max() / np.abs(ref[:, 0]).max(),
                      np.abs(dl - ref[:, 1]).max() / np.abs(ref[:, 1]).max())
    assert err[16][0] < 1e-8 and err[16][1] < 1e-7, err
    assert err[8][0] > 100 * err[16][0] and err[8][1] > 100 * err[16][1], err
