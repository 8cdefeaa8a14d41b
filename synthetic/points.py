"""Seeded space-time evaluation points for the representation formula."""
import numpy as np


def ball_points(n, radius=0.5, center=(0.0, 0.0, 0.0), seed=0):
    """n points uniform in a ball (rejection-free: direction x radius^(1/3))."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return np.asarray(center)[None, :] + d * r[:, None]


def box_points(n, lo=0.25, hi=0.75, seed=0):
    """n points uniform in the box [lo, hi]^3."""
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random((n, 3))


def space_time_points(x, t_lo=0.25, t_hi=0.75, seed=0):
    """Append a uniform time in [t_lo, t_hi] to each point: returns (P, 4) float64 (x, y, z, t)."""
    rng = np.random.default_rng(seed + 7919)
    t = t_lo + (t_hi - t_lo) * rng.random(len(x))
    return np.ascontiguousarray(np.column_stack([x, t]), dtype=np.float64)
