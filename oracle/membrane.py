"""Membrane constitutive forces on triangulated cells, float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.3 gives the force decomposition F_total = F_link + F_bend + F_area +
F_volume: link forces from spectrin stretching, bending rigidity, membrane
(area) incompressibility and quasi-incompressible volume, with a linear
response at small and a strongly non-linear response at large deformation,
relative to a stress-free rest state.  The explicit forms live in a
reference the paper does not reproduce, so this module uses the reading:

  link  (per edge, length L, rest L0, strain s = (L-L0)/L0):
        energy k_l L0 [s^2/2 - 1/2 ln(1 - s^2/tl^2)],  tl = 3
        -> force on i along (x_j - x_i)/L of size k_l (s + s/(tl^2 - s^2))
  bend  (per interior edge, dihedral theta, rest theta0, d = theta-theta0):
        energy k_b [d^2/2 - 1/2 ln(1 - d^2/tb^2)],  tb = pi/6
  area  (per cell, a = (A-A0)/A0):   energy k_a A0 a^2 / 2
  volume(per cell, v = (V-V0)/V0):   energy k_v V0 v^2 / 2
  plus a pole traction: +F/|P+| on each of the 32 vertices with the largest
  rest-frame x, -F/|P-| on the 32 with the smallest (ties: lower index).
Strain and angle arguments of the non-linear terms are clamped to +-0.99 of
their limits.  All forces are minus the exact gradient of these energies.

Dihedral convention: for an edge i->j in triangle t1 = (i, j, k) and j->i
in t2 = (j, i, l) (both counter-clockwise from outside),
theta = atan2((n1 x n2) . e, n1 . n2) with e the unit edge vector; theta > 0
on a convex fold.
"""
from __future__ import annotations

import math

import numpy as np

TAU_LINK = 3.0
TAU_BEND = math.pi / 6.0
CLAMP = 0.99
N_POLE = 32


class Topology:
    """Edges and dihedral hinges of a closed, consistently oriented mesh."""

    def __init__(self, tri: np.ndarray, n_vert: int):
        tri = np.asarray(tri, dtype=np.int64)
        self.tri = tri
        self.n_vert = n_vert
        directed = {}
        for t, (a, b, c) in enumerate(tri):
            for (p, q, r) in ((a, b, c), (b, c, a), (c, a, b)):
                directed[(p, q)] = (t, r)
        edges, hinges = [], []
        for (p, q), (t, r) in directed.items():
            if p < q:
                t2, s = directed[(q, p)]
                edges.append((p, q))
                hinges.append((p, q, r, s))
        order = np.lexsort((np.array(edges)[:, 1], np.array(edges)[:, 0]))
        self.edges = np.array(edges, dtype=np.int64)[order]
        self.hinges = np.array(hinges, dtype=np.int64)[order]   # (i, j, k, l)


def _norm(v):
    """Euclidean norm over the last axis, sqrt(v . v) (for complex input, the
    complex-step gradient, its analytic continuation)."""
    return np.sqrt((v * v).sum(axis=-1))


def _atan2(s, c):
    """atan2 of real arrays; for complex ones (the complex-step gradient) the
    real angle plus its first-order change, (c ds - s dc) / (s^2 + c^2),
    carried in the imaginary part."""
    if not (np.iscomplexobj(s) or np.iscomplexobj(c)):
        return np.arctan2(s, c)
    s, c = np.asarray(s, dtype=np.complex128), np.asarray(c, dtype=np.complex128)
    return np.arctan2(s.real, c.real) + 1j * (c.real * s.imag - s.real * c.imag) / (s.real ** 2 + c.real ** 2)


def _as_array(X):
    X = np.asarray(X)
    return X.astype(np.complex128 if np.iscomplexobj(X) else np.float64)


def triangle_normals(X, tri):
    """Unnormalised normals (x_j - x_i) x (x_k - x_i), per triangle."""
    a, b, c = X[..., tri[:, 0], :], X[..., tri[:, 1], :], X[..., tri[:, 2], :]
    return np.cross(b - a, c - a)


def area_volume(X, tri):
    """Cell surface area and enclosed volume (divergence theorem), per cell.

    X: [..., V, 3].  Volume uses the first vertex of each cell as origin.
    """
    N = triangle_normals(X, tri)
    A = 0.5 * _norm(N).sum(axis=-1)
    o = X[..., :1, :]
    a, b, c = X[..., tri[:, 0], :] - o, X[..., tri[:, 1], :] - o, X[..., tri[:, 2], :] - o
    V = (a * np.cross(b, c)).sum(axis=-1).sum(axis=-1) / 6.0
    return A, V


def dihedral(X, hinges):
    i, j, k, l = hinges.T
    xi, xj, xk, xl = X[..., i, :], X[..., j, :], X[..., k, :], X[..., l, :]
    e = xj - xi
    n1 = np.cross(xj - xi, xk - xi)
    n2 = np.cross(xi - xj, xl - xj)
    n1h = n1 / _norm(n1)[..., None]
    n2h = n2 / _norm(n2)[..., None]
    eh = e / _norm(e)[..., None]
    s = (np.cross(n1h, n2h) * eh).sum(axis=-1)
    c = (n1h * n2h).sum(axis=-1)
    return _atan2(s, c)


def edge_lengths(X, edges):
    return _norm(X[..., edges[:, 1], :] - X[..., edges[:, 0], :])


class RestState:
    """Rest lengths, rest angles, rest area and volume of the undeformed mesh,
    and the pole vertex sets used by the traction."""

    def __init__(self, rest_pos: np.ndarray, topo: Topology):
        X = np.asarray(rest_pos, dtype=np.float64)
        self.L0 = edge_lengths(X, topo.edges)
        self.theta0 = dihedral(X, topo.hinges)
        self.A0, self.V0 = (float(v) for v in area_volume(X, topo.tri))
        idx = np.arange(X.shape[0])
        self.p_plus = np.lexsort((idx, -X[:, 0]))[:N_POLE]
        self.p_minus = np.lexsort((idx, X[:, 0]))[:N_POLE]


def _g(x, lim):
    c = CLAMP * lim   # clamped on the real part (a clamped argument has zero derivative)
    x = np.where(np.real(x) > c, c, np.where(np.real(x) < -c, -c, x))
    return x + x / (lim * lim - x * x)


def link_forces(X, topo, rest):
    """F_link: -dE_link/dx, per vertex.  X [..., V, 3]."""
    i, j = topo.edges[:, 0], topo.edges[:, 1]
    d = X[..., j, :] - X[..., i, :]
    L = _norm(d)
    s = (L - rest.L0) / rest.L0
    f = (_g(s, TAU_LINK) / L)[..., None] * d          # force on i
    F = np.zeros_like(X)
    _scatter(F, i, f)
    _scatter(F, j, -f)
    return F


def bend_forces(X, topo, rest):
    """F_bend: -dE_bend/dx with the closed-form dihedral gradient."""
    i, j, k, l = topo.hinges.T
    xi, xj, xk, xl = X[..., i, :], X[..., j, :], X[..., k, :], X[..., l, :]
    e = xj - xi
    el2 = (e * e).sum(axis=-1)
    el = np.sqrt(el2)
    n1 = np.cross(xj - xi, xk - xi)
    n2 = np.cross(xi - xj, xl - xj)
    n1s = (n1 * n1).sum(axis=-1)
    n2s = (n2 * n2).sum(axis=-1)
    theta = dihedral(X, topo.hinges)
    # d theta / d x for the wing vertices: moving a wing along its face
    # normal flattens a convex fold.
    gk = -(el / n1s)[..., None] * n1
    gl = -(el / n2s)[..., None] * n2
    ak = ((xk - xi) * e).sum(axis=-1) / el2
    al = ((xl - xi) * e).sum(axis=-1) / el2
    gi = -(1.0 - ak)[..., None] * gk - (1.0 - al)[..., None] * gl
    gj = -ak[..., None] * gk - al[..., None] * gl
    m = -_g(theta - rest.theta0, TAU_BEND)[..., None]
    F = np.zeros_like(X)
    _scatter(F, i, m * gi)
    _scatter(F, j, m * gj)
    _scatter(F, k, m * gk)
    _scatter(F, l, m * gl)
    return F


def area_gradient(X, tri):
    """dA/dx per vertex: for triangle (v, j, k), 1/2 n_hat x (x_k - x_j)."""
    G = np.zeros_like(X)
    N = triangle_normals(X, tri)
    nh = N / _norm(N)[..., None]
    for r in range(3):
        v, j, k = tri[:, r], tri[:, (r + 1) % 3], tri[:, (r + 2) % 3]
        _scatter(G, v, 0.5 * np.cross(nh, X[..., k, :] - X[..., j, :]))
    return G


def volume_gradient(X, tri):
    """dV/dx per vertex: for triangle (v, j, k), 1/6 (x_j - o) x (x_k - o)."""
    G = np.zeros_like(X)
    o = X[..., :1, :]
    for r in range(3):
        v, j, k = tri[:, r], tri[:, (r + 1) % 3], tri[:, (r + 2) % 3]
        _scatter(G, v, np.cross(X[..., j, :] - o, X[..., k, :] - o) / 6.0)
    return G


def forces(X, k, topo, rest, traction=None, terms=("link", "bend", "area", "volume")):
    """Total membrane force per vertex for cells X [C, V, 3] with stiffness
    k [C, 4] = (link, bend, area, volume) and optional traction [C, 3]."""
    X = _as_array(X)
    k = _as_array(k)
    F = np.zeros(X.shape, dtype=np.result_type(X, k))
    if "link" in terms:
        F += k[:, 0, None, None] * link_forces(X, topo, rest)
    if "bend" in terms:
        F += k[:, 1, None, None] * bend_forces(X, topo, rest)
    if "area" in terms or "volume" in terms:
        A, V = area_volume(X, topo.tri)
        if "area" in terms:
            a = (A - rest.A0) / rest.A0
            F -= (k[:, 2] * a)[:, None, None] * area_gradient(X, topo.tri)
        if "volume" in terms:
            v = (V - rest.V0) / rest.V0
            F -= (k[:, 3] * v)[:, None, None] * volume_gradient(X, topo.tri)
    if traction is not None:
        t = np.asarray(traction, dtype=np.float64)
        F[:, rest.p_plus, :] += t[:, None, :] / len(rest.p_plus)
        F[:, rest.p_minus, :] -= t[:, None, :] / len(rest.p_minus)
    return F


def energy(X, k, topo, rest):
    """Total internal energy per cell whose negative gradient is `forces`
    (traction excluded), valid inside the clamp range."""
    X = np.asarray(X, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    s = (edge_lengths(X, topo.edges) - rest.L0) / rest.L0
    e_link = (rest.L0 * (0.5 * s * s - 0.5 * np.log(1.0 - s * s / TAU_LINK ** 2))).sum(axis=-1)
    d = dihedral(X, topo.hinges) - rest.theta0
    e_bend = (0.5 * d * d - 0.5 * np.log(1.0 - d * d / TAU_BEND ** 2)).sum(axis=-1)
    A, V = area_volume(X, topo.tri)
    a = (A - rest.A0) / rest.A0
    v = (V - rest.V0) / rest.V0
    return (k[:, 0] * e_link + k[:, 1] * e_bend + 0.5 * k[:, 2] * rest.A0 * a * a
            + 0.5 * k[:, 3] * rest.V0 * v * v)


def _scatter(F, idx, val):
    """F[..., idx, :] += val with repeated indices accumulated."""
    if F.ndim == 2:
        np.add.at(F, idx, val)
    else:
        np.add.at(F, (slice(None), idx), val)
