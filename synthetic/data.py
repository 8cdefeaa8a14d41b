"""Closed-form boundary data of the test problems (inputs, not part of the method).

* ``heat_kernel_solution``: u(x, t) = G_alpha(x - y*, t) with y* outside the domain.  It solves
  the heat equation with zero initial data, so it is the exact solution the discrete method must
  converge to (the paper's convergence experiment, Sec. 6.1).
* ``heat_kernel_flux``: its Neumann datum alpha du/dn(x, t) for an outward normal n.
* ``exp_solution``: u(x, t) = exp(alpha t + x.e) with |e| = 1, a heat solution with NONZERO
  initial data; it is used only as smooth synthetic Dirichlet data for timing and residual tests.
* ``nodal_samples``: coefficients in the space (p1 in space) x (p0 in time) obtained by sampling
  a function at the mesh vertices and interval midpoints (a synthetic data vector).
"""
import math
import numpy as np


def heat_kernel_solution(x, t, alpha, ystar):
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    r2 = np.sum((x - np.asarray(ystar)[None, :]) ** 2, axis=-1)
    out = np.zeros(np.broadcast(r2, t).shape)
    pos = t > 0
    tt = np.broadcast_to(t, out.shape)[pos]
    rr = np.broadcast_to(r2, out.shape)[pos]
    out[pos] = (4 * math.pi * alpha * tt) ** -1.5 * np.exp(-rr / (4 * alpha * tt))
    return out


def heat_kernel_flux(x, n, t, alpha, ystar):
    """alpha * grad_x G_alpha(x - y*, t) . n"""
    x = np.asarray(x, dtype=np.float64)
    d = x - np.asarray(ystar)[None, :]
    u = heat_kernel_solution(x, t, alpha, ystar)
    tt = np.maximum(np.asarray(t, dtype=np.float64), 1e-300)
    return alpha * u * (-np.sum(d * n, axis=-1) / (2 * alpha * tt))


def exp_solution(x, t, alpha, e=(1.0, 1.0, 1.0)):
    e = np.asarray(e, dtype=np.float64)
    e = e / np.linalg.norm(e)
    return np.exp(alpha * np.asarray(t) + np.asarray(x) @ e)


def nodal_samples(verts, n_t, T, fn):
    """(E_t, N_x) array of fn(vertex, midpoint of interval i)."""
    h = T / n_t
    out = np.empty((n_t, len(verts)))
    for i in range(n_t):
        out[i] = fn(verts, np.full(len(verts), (i + 0.5) * h))
    return out


class ExactSolution:
    """u = G_alpha(x - y*, t): value, Neumann datum on a triangle normal, for tests."""

    def __init__(self, alpha, ystar):
        self.alpha = alpha
        self.ystar = np.asarray(ystar, dtype=np.float64)

    def u(self, x, t):
        return heat_kernel_solution(x, t, self.alpha, self.ystar)

    def flux(self, x, n, t):
        return heat_kernel_flux(x, n, t, self.alpha, self.ystar)
