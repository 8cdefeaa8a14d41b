"""ctypes binding of oracle.c (test infrastructure only; see the package docstring)."""
import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force=False):
    """Compile oracle.c with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i32, f64 = ctypes.c_int, ctypes.c_double
        L.or_temporal.argtypes = [i32, _dp, _dp, i32, f64, _dp]
        L.or_temporal.restype = None
        L.or_blockfun.argtypes = [i32, _dp, _ip, i32, f64, f64, i32, _dp]
        L.or_blockfun.restype = None
        L.or_triangle_rule.argtypes = [i32, i32, _dp, _dp]
        L.or_ss_rule.argtypes = [i32, i32, _dp, _dp, _dp]
        L.or_gauss_legendre01.argtypes = [i32, _dp, _dp]
        L.or_pair_points.argtypes = [_dp, _ip, i32, i32, i32, _dp, _dp, _dp, _dp,
                                     ctypes.POINTER(ctypes.c_int)]
        L.or_assemble_d2.argtypes = [_dp, i32, _ip, i32, f64, f64, i32, i32, _dp]
        L.or_assemble_v11.argtypes = [_dp, i32, _ip, i32, f64, f64, i32, i32, _dp]
        L.or_pair_blocks.argtypes = [_dp, i32, _ip, i32, f64, f64, i32, i32, i32, i32, _dp, _dp]
        L.or_assemble.argtypes = [_dp, i32, _ip, i32, f64, f64, i32, i32, _ip, i32, i32, i32,
                                  _dp, _dp]
        L.or_assemble_plain.argtypes = [_dp, i32, _ip, i32, f64, f64, i32, i32, _ip, i32, i32,
                                        _dp, _dp]
        L.or_assemble_nonuniform.argtypes = [_dp, i32, _ip, i32, f64, _dp, i32, i32, _ip, i32,
                                             _dp, _dp]
        L.or_nu_blockfun.argtypes = [i32, _dp, _ip, _ip, i32, _dp, f64, _dp]
        L.or_nu_blockfun.restype = None
        L.or_repr.argtypes = [_dp, i32, _ip, i32, f64, f64, i32, _dp, _dp, _dp, i32, i32, i32,
                              _dp, _dp]
        L.or_repr_nonuniform.argtypes = [_dp, i32, _ip, i32, f64, _dp, i32, _dp, _dp, _dp, i32,
                                         i32, i32, _dp, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


_TEMPORAL = {"g1": 0, "F": 1, "Fn_rn": 2, "g1n_rn": 3}


def temporal(which, rho, delta, alpha):
    """G^{dtau} ('g1'), G^{dtau dt} ('F'), alpha dG^{dtau dt}/dn / (r.n) ('Fn_rn'),
    alpha dG^{dtau}/dn / (r.n) ('g1n_rn') at arrays rho, delta."""
    rho, delta = np.broadcast_arrays(_f64(rho), _f64(delta))
    rho, delta = _f64(rho.ravel()), _f64(delta.ravel())
    out = np.empty_like(rho)
    lib().or_temporal(_TEMPORAL[which], rho, delta, len(rho), float(alpha), out)
    return out


def blockfun(which, rho, d, h, alpha, tmode=0):
    """Exact per-point temporal block integrals: V^d(r) ('V'), K^d(r)/(r.n) ('K') or the
    hypersingular part D^{2,d}(r) ('D2', Sec. 3.3, closed form only).
    tmode 0: closed form for d <= 16, hat quadrature above; 1: closed form; 2: hat for d >= 2."""
    rho, d = np.broadcast_arrays(_f64(rho), np.asarray(d))
    rho, d = _f64(rho.ravel()), _i32(d.ravel())
    out = np.empty_like(rho)
    lib().or_blockfun({"V": 0, "K": 1, "D2": 2}[which], rho, d, len(rho), float(h), float(alpha),
                      int(tmode), out)
    return out


def triangle_rule(kind=0, order=7):
    """(barycentric (n, 3), weights (n,)) with weights summing to 1; kind 0 = Radon 7 point,
    kind 1 = collapsed Gauss with order^2 points."""
    n = 7 if kind == 0 else order * order
    lam, w = np.empty(3 * n), np.empty(n)
    c = lib().or_triangle_rule(kind, order, lam, w)
    return lam[:3 * c].reshape(c, 3), w[:c]


def ss_rule(cls, order):
    """Regularised rule on T x T for class cls (3 identical, 2 edge, 1 vertex):
    (x_hat (n, 2), y_hat (n, 2), w (n,)) with sum(w) = 1/4."""
    n = {3: 6, 2: 5, 1: 2}[cls] * order ** 4
    xh, yh, w = np.empty(2 * n), np.empty(2 * n), np.empty(n)
    c = lib().or_ss_rule(cls, order, xh, yh, w)
    return xh[:2 * c].reshape(c, 2), yh[:2 * c].reshape(c, 2), w[:c]


def gauss_legendre01(n):
    x, w = np.empty(n), np.empty(n)
    lib().or_gauss_legendre01(n, x, w)
    return x, w


def pair_points(verts, tris, a, b, ss_order=4):
    """Quadrature points of the ordered panel pair (test a, trial b): dict with x, y (n, 3),
    W (n,), phi (n, 3) (trial p1 basis at y for the trial panel's local vertices), cls."""
    verts, tris = _f64(verts), _i32(tris)
    cap = max(49, 6 * ss_order ** 4)
    x, y, W, phi = np.empty(3 * cap), np.empty(3 * cap), np.empty(cap), np.empty(3 * cap)
    cls = ctypes.c_int(0)
    n = lib().or_pair_points(verts.ravel(), tris.ravel(), a, b, ss_order, x, y, W, phi,
                             ctypes.byref(cls))
    return {"x": x[:3 * n].reshape(n, 3), "y": y[:3 * n].reshape(n, 3), "W": W[:n],
            "phi": phi[:3 * n].reshape(n, 3), "cls": cls.value}


def assemble(verts, tris, alpha, T, n_t, rows=None, ss_order=4, method="direct", tmode=0):
    """Blocks V_h^d (n_t, len(rows), E_x) and K_h^d (n_t, len(rows), N_x) for the test rows."""
    verts, tris = _f64(verts), _i32(tris)
    ne, nv = len(tris), len(verts)
    rows = _i32(np.arange(ne) if rows is None else rows)
    V = np.empty((n_t, len(rows), ne))
    K = np.empty((n_t, len(rows), nv))
    rc = lib().or_assemble(verts.ravel(), nv, tris.ravel(), ne, float(alpha), float(T), n_t,
                           ss_order, rows, len(rows), 0 if method == "direct" else 1, tmode,
                           V, K)
    if rc != 0:
        raise ValueError("or_assemble failed (%d)" % rc)
    return V, K


def assemble_plain(verts, tris, alpha, T, n_t, rows=None, ss_order=4, threads=0):
    """The method as the paper runs it on a CPU (Sec. 5.1): double precision, level order,
    OpenMP over test rows (threads > 0 fixes the team size).  The timed CPU baseline; its blocks
    at large d carry the rounding of the second differences, so it is not a parity reference.
    Same shapes as assemble()."""
    verts, tris = _f64(verts), _i32(tris)
    ne, nv = len(tris), len(verts)
    rows = _i32(np.arange(ne) if rows is None else rows)
    V = np.empty((n_t, len(rows), ne))
    K = np.empty((n_t, len(rows), nv))
    rc = lib().or_assemble_plain(verts.ravel(), nv, tris.ravel(), ne, float(alpha), float(T), n_t,
                                 ss_order, rows, len(rows), int(threads), V, K)
    if rc != 0:
        raise ValueError("or_assemble_plain failed (%d)" % rc)
    return V, K


def assemble_nonuniform(verts, tris, alpha, t_nodes, rows=None, ss_order=4):
    """Blocks on the non-uniform time grid t_nodes (0 = t_0 < ... < t_nt): V (nb, len(rows), E_x)
    and K (nb, len(rows), N_x), nb = nt (nt + 1) / 2, block (k, i) (0 <= i <= k < nt) at index
    k (k + 1) / 2 + i."""
    verts, tris, tn = _f64(verts), _i32(tris), _f64(t_nodes)
    ne, nv, nt = len(tris), len(verts), len(tn) - 1
    rows = _i32(np.arange(ne) if rows is None else rows)
    nb = nt * (nt + 1) // 2
    V = np.empty((nb, len(rows), ne))
    K = np.empty((nb, len(rows), nv))
    rc = lib().or_assemble_nonuniform(verts.ravel(), nv, tris.ravel(), ne, float(alpha), tn, nt,
                                      ss_order, rows, len(rows), V, K)
    if rc != 0:
        raise ValueError("or_assemble_nonuniform failed (%d)" % rc)
    return V, K


def nu_blockfun(which, rho, k, i, t_nodes, alpha):
    """Per-point block integrals on a grid: V^{k,i}(rho) ('V') or K^{k,i}(rho) / (r . n) ('K')."""
    rho, k, i = np.broadcast_arrays(_f64(rho), np.asarray(k), np.asarray(i))
    rho, k, i = _f64(rho.ravel()), _i32(k.ravel()), _i32(i.ravel())
    out = np.empty_like(rho)
    lib().or_nu_blockfun({"V": 0, "K": 1}[which], rho, k, i, len(rho), _f64(t_nodes), float(alpha),
                         out)
    return out


def repr_eval(verts, tris, alpha, T, n_t, w, u, pts, rule_kind=0, rule_order=7):
    """Single-layer potential V~w and double-layer potential Wu at space-time points (P, 4).
    The representation formula is u(x, t) = sl - dl."""
    verts, tris = _f64(verts), _i32(tris)
    w, u, pts = _f64(w), _f64(u), _f64(pts)
    P = len(pts)
    sl, dl = np.empty(P), np.empty(P)
    rc = lib().or_repr(verts.ravel(), len(verts), tris.ravel(), len(tris), float(alpha),
                       float(T), n_t, w.ravel(), u.ravel(), pts.ravel(), P, rule_kind,
                       rule_order, sl, dl)
    if rc != 0:
        raise ValueError("or_repr failed")
    return sl, dl


def repr_eval_nonuniform(verts, tris, alpha, t_nodes, w, u, pts, rule_kind=0, rule_order=7):
    """V~w and Wu at space-time points (P, 4) on the non-uniform grid t_nodes (0 = t_0 < ... <
    t_nt); w (nt, E_x) and u (nt, N_x) hold one row per interval [t_i, t_{i+1}]."""
    verts, tris, tn = _f64(verts), _i32(tris), _f64(t_nodes)
    w, u, pts = _f64(w), _f64(u), _f64(pts)
    P = len(pts)
    sl, dl = np.empty(P), np.empty(P)
    rc = lib().or_repr_nonuniform(verts.ravel(), len(verts), tris.ravel(), len(tris), float(alpha),
                                  tn, len(tn) - 1, w.ravel(), u.ravel(), pts.ravel(), P, rule_kind,
                                  rule_order, sl, dl)
    if rc != 0:
        raise ValueError("or_repr_nonuniform failed")
    return sl, dl


def assemble_d2(verts, tris, alpha, T, n_t, ss_order=4):
    """Blocks D_h^{2,d} (n_t, N_x, N_x) of the hypersingular operator's second part (Sec. 3.3):
    p1 x p1 with n(x) . n(y) and the kernel D^{2,d}, every ordered panel pair, the same rules as
    for V and K."""
    verts, tris = _f64(verts), _i32(tris)
    ne, nv = len(tris), len(verts)
    D2 = np.empty((n_t, nv, nv))
    rc = lib().or_assemble_d2(verts.ravel(), nv, tris.ravel(), ne, float(alpha), float(T), n_t,
                              ss_order, D2)
    if rc != 0:
        raise ValueError("or_assemble_d2 failed (%d)" % rc)
    return D2


def assemble_v11(verts, tris, alpha, T, n_t, ss_order=4):
    """Blocks V_h^{11,d} (n_t, N_x, N_x): the single layer between p1 test and p1 trial functions
    (the matrix of the operator preconditioner for D_h, Sec. 6.1), same rules as V_h."""
    verts, tris = _f64(verts), _i32(tris)
    ne, nv = len(tris), len(verts)
    V11 = np.empty((n_t, nv, nv))
    rc = lib().or_assemble_v11(verts.ravel(), nv, tris.ravel(), ne, float(alpha), float(T), n_t,
                               ss_order, V11)
    if rc != 0:
        raise ValueError("or_assemble_v11 failed (%d)" % rc)
    return V11


def pair_blocks(verts, tris, alpha, T, n_t, a, b, ss_order=4):
    """One ordered panel pair (test a, trial b): V (n_t,) = V_h^d[a][b] and K (n_t, 3) = the
    contributions of panel b to row a of K_h^d through its local vertices."""
    verts, tris = _f64(verts), _i32(tris)
    V = np.empty(n_t)
    K = np.empty((n_t, 3))
    rc = lib().or_pair_blocks(verts.ravel(), len(verts), tris.ravel(), len(tris), float(alpha),
                              float(T), n_t, ss_order, int(a), int(b), V, K.ravel())
    if rc != 0:
        raise ValueError("or_pair_blocks failed (%d)" % rc)
    return V, K
