"""Closed triangulated surfaces used as workloads (outward, counter-clockwise seen from outside).

Every generator returns ``(verts, tris)``: ``verts`` is a float64 array (N_x, 3) and ``tris``
an int32 array (E_x, 3) whose vertex order is counter-clockwise when seen from outside the
enclosed volume, so that (v1 - v0) x (v2 - v0) points outward.

Workloads (all seeded or deterministic):

* ``cube(n)``: each face of an axis-aligned cube cut into n x n squares, each square split along
  its (i, j) -> (i+1, j+1) diagonal.  n = 4 on the unit cube gives 192 triangles / 98 vertices,
  n = 16 gives 3072 / 1538 (the paper's 32-triangles-per-face coarse mesh is n = 4 on (-1, 1)^3).
* ``cube4(n)``: each square split into four triangles through its centre; n = 16 gives 6144
  triangles / 3074 vertices.
* ``icosphere(level)``: icosahedron refined by edge midpoints and projected to the sphere;
  level 3 gives 1280 triangles / 642 vertices.
* ``cubed_sphere_ellipsoid(n, axes)``: cube(n) on (-1, 1)^3 projected to the unit sphere and
  scaled by the semi-axes; 12 n^2 triangles.
* ``tetrahedron()``, ``octahedron()``, ``two_separated_triangles()``: tiny edge cases.
"""
import numpy as np

# Each cube face: fixed axis, side (0 = low, 1 = high) and the two in-face axes (u, v) ordered
# so that e_u x e_v is the outward normal of that face.
_FACES = (
    (0, 1, 1, 2), (0, 0, 2, 1),
    (1, 1, 2, 0), (1, 0, 0, 2),
    (2, 1, 0, 1), (2, 0, 1, 0),
)


def _finish(keys_to_idx, coords, tris):
    verts = np.asarray(coords, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int32)
    return verts, tris


def cube(n, lo=0.0, hi=1.0):
    """Cube surface [lo, hi]^3 with n x n squares per face, two triangles per square."""
    if n < 1:
        raise ValueError("n must be >= 1")
    index, coords, tris = {}, [], []

    def vid(key):
        if key not in index:
            index[key] = len(coords)
            coords.append([lo + (hi - lo) * k / n for k in key])
        return index[key]

    for axis, side, ua, va in _FACES:
        for i in range(n):
            for j in range(n):
                def p(a, b):
                    key = [0, 0, 0]
                    key[axis] = side * n
                    key[ua] = a
                    key[va] = b
                    return vid(tuple(key))
                p00, p10, p11, p01 = p(i, j), p(i + 1, j), p(i + 1, j + 1), p(i, j + 1)
                tris.append((p00, p10, p11))
                tris.append((p00, p11, p01))
    return _finish(index, coords, tris)


def cube4(n, lo=0.0, hi=1.0):
    """Cube surface with n x n squares per face, each split into 4 triangles through its centre."""
    if n < 1:
        raise ValueError("n must be >= 1")
    index, coords, tris = {}, [], []
    m = 2 * n

    def vid(key):
        if key not in index:
            index[key] = len(coords)
            coords.append([lo + (hi - lo) * k / m for k in key])
        return index[key]

    for axis, side, ua, va in _FACES:
        for i in range(n):
            for j in range(n):
                def p(a, b):
                    key = [0, 0, 0]
                    key[axis] = side * m
                    key[ua] = a
                    key[va] = b
                    return vid(tuple(key))
                p00, p10 = p(2 * i, 2 * j), p(2 * i + 2, 2 * j)
                p11, p01 = p(2 * i + 2, 2 * j + 2), p(2 * i, 2 * j + 2)
                c = p(2 * i + 1, 2 * j + 1)
                tris += [(p00, p10, c), (p10, p11, c), (p11, p01, c), (p01, p00, c)]
    return _finish(index, coords, tris)


def icosphere(level, radius=1.0):
    """Icosahedron refined ``level`` times by edge midpoints, vertices projected to the sphere."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                pm = verts[a] + verts[b]
                verts.append(pm / np.linalg.norm(pm))
                mid[key] = len(verts) - 1
            return mid[key]
        new = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new
    verts = radius * np.array(verts)
    return verts.astype(np.float64), np.asarray(faces, dtype=np.int32)


def cubed_sphere_ellipsoid(n, axes=(1.0, 1.0, 1.0)):
    """cube(n) on (-1, 1)^3 projected radially to the unit sphere, then scaled by ``axes``."""
    verts, tris = cube(n, -1.0, 1.0)
    verts = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    return verts * np.asarray(axes, dtype=np.float64)[None, :], tris


def tetrahedron():
    """Regular-ish tetrahedron: every pair of faces shares an edge."""
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    tris = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)
    return verts, tris


def octahedron(radius=1.0):
    """Octahedron: identical, edge-, vertex-sharing and (antipodal) separated face pairs."""
    verts = radius * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1],
                               [0, 0, -1]], dtype=np.float64)
    tris = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                     [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    return verts, tris


def two_separated_triangles(gap=0.5):
    """Two parallel, non-touching triangles facing each other (not a closed surface)."""
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0],
                      [0.2, 0.1, gap], [0.1, 1.1, gap], [1.0, 0.3, gap]], dtype=np.float64)
    tris = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    return verts, tris


def mesh_summary(verts, tris):
    """Counts and the Euler characteristic (2 for a closed genus-0 surface)."""
    tris = np.asarray(tris)
    edges = set()
    for a, b, c in tris:
        for p, q in ((a, b), (b, c), (c, a)):
            edges.add((min(p, q), max(p, q)))
    return {"n_verts": len(verts), "n_tris": len(tris), "n_edges": len(edges),
            "euler": len(verts) - len(edges) + len(tris)}
