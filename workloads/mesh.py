"""Triangulated red-blood-cell surface mesh (input generator).

The paper represents each cell by a triangulated membrane whose vertices
move in a Lagrangian frame (Sec. 2.3).  It gives no mesh recipe, so this
module builds one: an icosphere refined by edge-midpoint subdivision and
mapped onto the Evans-Fung biconcave profile.  Diameter and thickness of the
result fall inside the ranges the paper quotes for an undeformed RBC
(6-8 um across, 2-3 um thick; Sec. 1) at 0.5 um per lattice unit.

This module only produces geometry used as input.  It holds none of the
method's arithmetic (no forces, no rest-state quantities): the oracle and
the device library each derive edge lengths, angles, area and volume from
the positions returned here on their own.
"""
from __future__ import annotations

import numpy as np

# Evans-Fung profile coefficients for z(s) = (a/2) * sqrt(1-s) * (c0 + c1 s + c2 s^2),
# s = (r/a)^2, a = cell radius (literature values of the biconcave fit).
EF_C0 = 0.2072
EF_C1 = 2.0026
EF_C2 = -1.1228


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def icosphere(level: int):
    """Unit icosphere after `level` midpoint subdivisions.

    Returns (vertices float64 [V,3], triangles int32 [T,3]); triangles are
    counter-clockwise seen from outside, so (x1-x0) x (x2-x0) points outward.
    Level 3 gives 642 vertices and 1280 triangles.
    """
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    faces = f.tolist()
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            if key in cache:
                return cache[key]
            p = np.add(verts[a], verts[b]) * 0.5
            p = p / np.linalg.norm(p)
            verts.append(tuple(p))
            cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        faces = nf
    V = np.array(verts, dtype=np.float64)
    T = np.array(faces, dtype=np.int32)
    # orient every face outward (the sphere is convex and centred at 0)
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    c = V[T].mean(axis=1)
    flip = (n * c).sum(axis=1) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return V, T


def evans_fung(unit_sphere: np.ndarray, radius: float = 8.0) -> np.ndarray:
    """Map unit-sphere points onto the biconcave Evans-Fung surface.

    X = a x, Y = a y, Z = (a/2) z (c0 + c1 s + c2 s^2) with s = x^2 + y^2.
    The disk lies in the x-y plane; z is the thin axis.
    """
    x, y, z = unit_sphere[:, 0], unit_sphere[:, 1], unit_sphere[:, 2]
    s = x * x + y * y
    a = float(radius)
    return np.stack([a * x, a * y, 0.5 * a * z * (EF_C0 + EF_C1 * s + EF_C2 * s * s)], axis=1)


def rbc_mesh(level: int = 3, diameter: float = 16.0):
    """Biconcave RBC mesh: (rest positions float64 [V,3] centred at 0, triangles int32 [T,3])."""
    v, t = icosphere(level)
    return evans_fung(v, 0.5 * diameter), t


def sphere_mesh(level: int = 2, radius: float = 4.0):
    """Icosphere of the given radius (used by convex-geometry pins)."""
    v, t = icosphere(level)
    return v * radius, t
