"""Oracle downstream of the blocks (test infrastructure only), plain float64 numpy/scipy.

* mass matrices M_x (p0 test x p1 trial) and the p1 mass matrix          (Sec. 3.4)
* L2 projections into X^{1,0} (Dirichlet data) and X^{0,0} (Neumann data)  (Sec. 3.4, Sec. 6.1)
* block lower-triangular Toeplitz apply y^k = sum_{d<=k} A^d x^{k-d}      (Sec. 3.1, eq. for V_h w)
* Dirichlet right-hand side (1/2 M_h + K_h) g                             (Sec. 3.4)
* time marching (block forward substitution with a Cholesky factor of V^0) and unrestarted
  GMRES with zero initial guess (the paper solves with FGMRES to relative accuracy 1e-8, Sec. 6.1)
* relative L2(Sigma_h) errors and the relative l2 point error              (Sec. 6.1)
* surface curls of the p1 basis, D_h^{1,d} = T^T (alpha^2 V^d (x) I_3) T,
  D_h = D_h^1 + D_h^2 and the Neumann right-hand side (1/2 M_h^T - K_h^T) h  (Sec. 3.3, 3.4)

Vectors are time-major: row i of an (E_t, n) array holds the coefficients of interval i+1.
"""
import numpy as np
import scipy.linalg

from . import core


def geometry(verts, tris):
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(v1 - v0, v2 - v0)
    nn = np.linalg.norm(cr, axis=1)
    return 0.5 * nn, cr / nn[:, None]


def mass_p0p1(verts, tris):
    """M_x[l, j] = int phi^0_l phi^1_j = area_l / 3 for the three vertices j of panel l."""
    area, _ = geometry(verts, tris)
    M = np.zeros((len(tris), len(verts)))
    for k in range(3):
        np.add.at(M, (np.arange(len(tris)), tris[:, k]), area / 3.0)
    return M


def mass_p1p1(verts, tris):
    area, _ = geometry(verts, tris)
    M = np.zeros((len(verts), len(verts)))
    for a in range(3):
        for b in range(3):
            np.add.at(M, (tris[:, a], tris[:, b]), area * (2.0 if a == b else 1.0) / 12.0)
    return M


def _space_time_nodes(verts, tris, n_t, T, q_space, q_time):
    lam, wq = core.triangle_rule(1, q_space)
    tq, wt = core.gauss_legendre01(q_time)
    v = verts[tris]                                  # (E, 3, 3)
    x = np.einsum("qk,ekc->eqc", lam, v)              # (E, nq, 3)
    h = T / n_t
    times = (np.arange(n_t)[:, None] + tq[None, :]) * h  # (E_t, nqt)
    return lam, wq, x, times, wt * h


def project_p1p0(verts, tris, n_t, T, fn, q_space=8, q_time=8):
    """Coefficients (E_t, N_x) of the L2(Sigma_h) projection of fn(x (n,3), t (n,)) into X^{1,0}."""
    area, _ = geometry(verts, tris)
    lam, wq, x, times, wt = _space_time_nodes(verts, tris, n_t, T, q_space, q_time)
    Mc = scipy.linalg.cho_factor(mass_p1p1(verts, tris))  # one Cholesky factor for every step
    E, nq = x.shape[0], x.shape[1]
    out = np.empty((n_t, len(verts)))
    h = T / n_t
    xf = x.reshape(-1, 3)
    for i in range(n_t):
        rhs = np.zeros(len(verts))
        for a, t in enumerate(times[i]):
            g = fn(xf, np.full(len(xf), t)).reshape(E, nq)
            for k in range(3):
                np.add.at(rhs, tris[:, k], wt[a] * area * (g * (wq * lam[:, k])[None, :]).sum(1))
        out[i] = scipy.linalg.cho_solve(Mc, rhs / h)
    return out


def project_p0p0(verts, tris, n_t, T, fn, q_space=8, q_time=8):
    """Coefficients (E_t, E_x) of the L2 projection of fn(x, n, t) into X^{0,0} (panel means)."""
    area, normal = geometry(verts, tris)
    lam, wq, x, times, wt = _space_time_nodes(verts, tris, n_t, T, q_space, q_time)
    E, nq = x.shape[0], x.shape[1]
    nrm = np.repeat(normal, nq, axis=0)
    h = T / n_t
    out = np.empty((n_t, E))
    for i in range(n_t):
        acc = np.zeros(E)
        for a, t in enumerate(times[i]):
            g = fn(x.reshape(-1, 3), nrm, np.full(E * nq, t)).reshape(E, nq)
            acc += wt[a] * (g * wq[None, :]).sum(1)
        out[i] = acc / h
    return out


def l2_error_p0(verts, tris, n_t, T, coeffs, fn, q_space=8, q_time=8):
    """Relative L2(Sigma_h) error of the p0 x p0 function `coeffs` against fn(x, n, t)."""
    area, normal = geometry(verts, tris)
    lam, wq, x, times, wt = _space_time_nodes(verts, tris, n_t, T, q_space, q_time)
    E, nq = x.shape[0], x.shape[1]
    nrm = np.repeat(normal, nq, axis=0)
    num = den = 0.0
    for i in range(n_t):
        for a, t in enumerate(times[i]):
            g = fn(x.reshape(-1, 3), nrm, np.full(E * nq, t)).reshape(E, nq)
            e = g - coeffs[i][:, None]
            num += wt[a] * np.sum(area[:, None] * wq[None, :] * e * e)
            den += wt[a] * np.sum(area[:, None] * wq[None, :] * g * g)
    return float(np.sqrt(num / den))


def toeplitz_apply(blocks, x):
    """y^k = sum_{d=0}^{k} A^d x^{k-d}; blocks (E_t, R, C), x (E_t, C) -> (E_t, R)."""
    n_t = blocks.shape[0]
    y = np.zeros((n_t, blocks.shape[1]))
    for k in range(n_t):
        for d in range(k + 1):
            y[k] += blocks[d] @ x[k - d]
    return y


def rhs_dirichlet(K, Mx, g, h):
    """(1/2 M_h + K_h) g with M_h = h blockdiag(M_x)."""
    return 0.5 * h * (g @ Mx.T) + toeplitz_apply(K, g)


def time_march(V, b):
    """Solve V_h w = b by block forward substitution with an LU factorisation of V^0.
    (V_h^0 is symmetric positive definite in exact arithmetic, but the assembled block is
    symmetric only up to the regularised rules' error, so a Cholesky factor, which reads one
    triangle, would solve a different matrix.)"""
    n_t = V.shape[0]
    lu = scipy.linalg.lu_factor(V[0])
    w = np.zeros_like(b)
    for k in range(n_t):
        r = b[k].copy()
        for d in range(1, k + 1):
            r -= V[d] @ w[k - d]
        w[k] = scipy.linalg.lu_solve(lu, r)
    return w


def gmres(apply, b, tol=1e-8, maxit=500):
    """Unrestarted GMRES (modified Gram-Schmidt, Givens rotations), zero initial guess.
    Returns (x, iterations, relative residual estimate)."""
    shape = b.shape
    b = b.ravel()
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(shape), 0, 0.0
    n = len(b)
    m = min(maxit, n)
    Q = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs, sn = np.zeros(m), np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    Q[0] = b / beta
    it = 0
    for j in range(m):
        w = apply(Q[j].reshape(shape)).ravel()
        for i in range(j + 1):
            H[i, j] = Q[i] @ w
            w = w - H[i, j] * Q[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0:
            Q[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        r = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / r, H[j + 1, j] / r
        H[j, j] = r
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        it = j + 1
        if abs(g[j + 1]) / beta <= tol:
            break
    y = scipy.linalg.solve_triangular(H[:it, :it], g[:it])
    x = Q[:it].T @ y
    return x.reshape(shape), it, abs(g[it]) / beta


def relative_l2(a, b):
    """sqrt(sum |a - b|^2) / sqrt(sum |a|^2)"""
    return float(np.linalg.norm(a - b) / np.linalg.norm(a))


def block_rel_error(A, B):
    """Per-block max-norm error relative to the block max: e_d = max|A^d - B^d| / max|A^d|."""
    A = np.asarray(A)
    B = np.asarray(B)
    num = np.abs(A - B).reshape(A.shape[0], -1).max(1)
    den = np.abs(A).reshape(A.shape[0], -1).max(1)
    return num / np.where(den > 0, den, 1.0)


def surface_curls(verts, tris):
    """curl_Gamma of the three local p1 basis functions on each panel, (E, 3 local, 3 coords):
    curl = n x grad_Gamma lambda_k = (x_{k+1} - x_{k+2}) / (2 area) (Sec. 2, surface curl)."""
    v = verts[tris]                                   # (E, 3, 3)
    area, _ = geometry(verts, tris)
    out = np.empty_like(v)
    for k in range(3):
        out[:, k, :] = (v[:, (k + 1) % 3, :] - v[:, (k + 2) % 3, :]) / (2.0 * area[:, None])
    return out


def assemble_d1(V, verts, tris, alpha):
    """D_h^{1,d} = T^T (alpha^2 V^d (x) I_3) T with T_o[m, j] the o-th component of the surface
    curl of phi^1_j on panel m (Sec. 3.3, eq. for D_h^{1,d})."""
    curls = surface_curls(verts, tris)
    ne, nv = len(tris), len(verts)
    D1 = np.zeros((V.shape[0], nv, nv))
    for o in range(3):
        To = np.zeros((ne, nv))
        for k in range(3):
            np.add.at(To, (np.arange(ne), tris[:, k]), curls[:, k, o])
        for d in range(V.shape[0]):
            D1[d] += alpha * alpha * (To.T @ V[d] @ To)
    return D1


def rhs_neumann(K, Mx, psi, h):
    """(1/2 M_h^T - K_h^T) psi with the blockwise transposes (Sec. 3.4, the Neumann system; the
    remark on K_T'): M_h = h blockdiag(M_x), K^T = the blocks K^d transposed one by one."""
    return 0.5 * h * (psi @ Mx) - toeplitz_apply(np.ascontiguousarray(K.transpose(0, 2, 1)), psi)


def l2_error_p1p0(verts, tris, n_t, T, coeffs, fn, q_space=8, q_time=8):
    """Relative L2(Sigma_h) error of the p1 (space) x p0 (time) function `coeffs` (E_t, N_x)
    against fn(x, t)."""
    area, _ = geometry(verts, tris)
    lam, wq, x, times, wt = _space_time_nodes(verts, tris, n_t, T, q_space, q_time)
    E, nq = x.shape[0], x.shape[1]
    num = den = 0.0
    for i in range(n_t):
        uh = np.einsum("qk,ek->eq", lam, coeffs[i][tris])
        for a, t in enumerate(times[i]):
            g = fn(x.reshape(-1, 3), np.full(E * nq, t)).reshape(E, nq)
            e = g - uh
            num += wt[a] * np.sum(area[:, None] * wq[None, :] * e * e)
            den += wt[a] * np.sum(area[:, None] * wq[None, :] * g * g)
    return float(np.sqrt(num / den))
