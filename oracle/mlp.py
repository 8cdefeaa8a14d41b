"""Oracle of the learned preconditioner's arithmetic (test infrastructure only), float64 numpy.

Not from the paper: the paper's solver is FGMRES without a learned component (Sec. 6.1).  This
module restates, plainly, what the library's kernels compute for it:
* the 3-layer tanh MLP (W1 [H][I], b1, W2 [H][H], b2, W3 [O][H], b3) forward and backward;
* the sparse-approximate-inverse training loss of a row, y^T G y - 2 a^T y + 1, with
  G = V^0[J,:] V^0[J,:]^T / V^0[l,l]^2 and a = V^0[J,l] / V^0[l,l]  (J = the row's pattern);
* one Adam step.
"""
import numpy as np


def unpack(params, n_in, n_h, n_out):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + n_h * n_in].reshape(n_h, n_in); o += n_h * n_in
    b1 = p[o:o + n_h]; o += n_h
    W2 = p[o:o + n_h * n_h].reshape(n_h, n_h); o += n_h * n_h
    b2 = p[o:o + n_h]; o += n_h
    W3 = p[o:o + n_out * n_h].reshape(n_out, n_h); o += n_out * n_h
    b3 = p[o:o + n_out]; o += n_out
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def forward(params, x, n_in, n_h, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, n_h, n_out)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3, (x, h1, h2)


def backward(params, cache, dy, n_in, n_h, n_out):
    """Gradient of sum(dy * y) w.r.t. the parameters (same flat layout)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, n_h, n_out)
    x, h1, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    dW3, db3 = dy.T @ h2, dy.sum(0)
    dz2 = (dy @ W3) * (1 - h2 * h2)
    dW2, db2 = dz2.T @ h1, dz2.sum(0)
    dz1 = (dz2 @ W2) * (1 - h1 * h1)
    dW1, db1 = dz1.T @ x, dz1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def row_loss(y, G, a):
    """Per-row y^T G y - 2 a^T y + 1 and the gradient of the batch mean w.r.t. y."""
    y = np.asarray(y, dtype=np.float64)
    Gy = np.einsum("bst,bt->bs", G, y)
    L = np.einsum("bs,bs->b", y, Gy) - 2 * np.einsum("bs,bs->b", a, y) + 1.0
    return L, 2 * (Gy - a) / len(y)


def spai_normal_equations(V0, cols):
    """G [E][S][S], a [E][S] of every row (absent slots: identity / zero) and the exact weights."""
    E, S = cols.shape
    G = np.zeros((E, S, S))
    a = np.zeros((E, S))
    y = np.zeros((E, S))
    for l in range(E):
        J = cols[l]
        ok = J >= 0
        s = V0[l, l]
        R = V0[J[ok], :] / s
        Gs = np.eye(S)
        Gs[np.ix_(ok, ok)] = R @ R.T
        G[l] = Gs
        a[l, ok] = V0[J[ok], l] / s
        y[l] = np.linalg.solve(Gs, a[l])
    return G, a, y


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps), m, v
