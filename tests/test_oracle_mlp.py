"""Pins of the oracle MLP: the backward pass equals finite differences of the forward pass, the
loss gradient equals finite differences of the loss, and the exact weights minimise the loss."""
import numpy as np

from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    I, H, O, Bt = 7, 9, 4, 5
    n = H * I + H + H * H + H + O * H + O
    p = rng.normal(scale=0.4, size=n)
    x = rng.normal(size=(Bt, I))
    dy = rng.normal(size=(Bt, O))
    y, cache = mlp.forward(p, x, I, H, O)
    g = mlp.backward(p, cache, dy, I, H, O)
    eps = 1e-6
    for k in rng.choice(n, 40, replace=False):
        e = np.zeros(n)
        e[k] = eps
        fd = (np.sum(dy * mlp.forward(p + e, x, I, H, O)[0]) -
              np.sum(dy * mlp.forward(p - e, x, I, H, O)[0])) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd))


def test_loss_gradient_and_minimiser():
    rng = np.random.default_rng(1)
    Bt, S = 3, 6
    R = rng.normal(size=(Bt, S, 20))
    G = np.einsum("bsj,btj->bst", R, R) + np.eye(S)
    a = rng.normal(size=(Bt, S))
    y = rng.normal(size=(Bt, S))
    L, dy = mlp.row_loss(y, G, a)
    eps = 1e-6
    for b in range(Bt):
        for s in range(S):
            e = np.zeros_like(y)
            e[b, s] = eps
            fd = (mlp.row_loss(y + e, G, a)[0].mean() - mlp.row_loss(y - e, G, a)[0].mean()) / (2 * eps)
            assert abs(fd - dy[b, s]) < 1e-7
    ystar = np.linalg.solve(G, a[..., None])[..., 0]
    assert np.all(mlp.row_loss(ystar, G, a)[0] <= L)


def test_spai_normal_equations_are_the_row_residual():
    """y^T G y - 2 a^T y + 1 = || (M V0)_l - e_l ||^2 for M[l, J] = y / V0[l,l]."""
    rng = np.random.default_rng(2)
    E = 12
    A = rng.normal(size=(E, E)) + E * np.eye(E)
    cols = np.full((E, 4), -1, dtype=np.int32)
    for l in range(E):
        cols[l, :3] = [l, (l + 1) % E, (l + 5) % E]
    G, a, y = mlp.spai_normal_equations(A, cols)
    yr = rng.normal(size=(E, 4))
    yr[:, 3] = 0.0
    for l in range(E):
        M = np.zeros(E)
        M[cols[l, :3]] = yr[l, :3] / A[l, l]
        direct = np.sum((M @ A - np.eye(E)[l]) ** 2)
        assert abs(mlp.row_loss(yr[l:l + 1], G[l:l + 1], a[l:l + 1])[0][0] - direct) < 1e-10
