"""Lattice sites inside the cells, float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

The cytosol is five times more viscous than plasma (Sec. 1), and stiffened
cells are modelled by scaling, among others, the internal viscosity ratio
(Sec. 3.4).  Reading: sites inside a cell relax with the viscosity ratio
lambda times the plasma viscosity, tau_in = 1/2 + lambda (tau - 1/2).  A
site is inside a cell by ray parity along z: the vertical line through the
site's (x, y) crosses the closed membrane at heights z_1 < z_2 < ...; the
site is inside when it lies strictly between z_(2k-1) and z_(2k).  A point
that falls exactly on a projected edge is counted by one of the two
triangles sharing it: after orienting each triangle counter-clockwise in the
(x, y) projection, an edge P -> Q keeps its boundary points when
Q.y > P.y, or Q.y == P.y and Q.x < P.x.  Periodic axes wrap; sites beyond a
wall are not marked.
"""
from __future__ import annotations

import numpy as np

WALL = 1


def _edge_in(px, py, qx, qy, x, y):
    """Point (x, y) on the inner side of, or on the kept part of, edge P -> Q
    of a counter-clockwise triangle."""
    w = (qx - px) * (y - py) - (qy - py) * (x - px)
    keep = (qy > py) | ((qy == py) & (qx < px))
    return (w > 0) | ((w == 0) & keep)


def crossings(V: np.ndarray, tri: np.ndarray, x: np.ndarray, y: np.ndarray):
    """Heights at which the vertical lines through (x[j], y[j]) cross the
    surface (V [nv, 3], triangles tri [nt, 3]).  Returns a list of sorted
    arrays, one per line."""
    a, b, c = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    ccw = area2 > 0
    b2 = np.where(ccw[:, None], b, c)
    c2 = np.where(ccw[:, None], c, b)
    A = np.abs(area2)
    X = x[:, None]
    Y = y[:, None]
    inside = (_edge_in(a[:, 0], a[:, 1], b2[:, 0], b2[:, 1], X, Y)
              & _edge_in(b2[:, 0], b2[:, 1], c2[:, 0], c2[:, 1], X, Y)
              & _edge_in(c2[:, 0], c2[:, 1], a[:, 0], a[:, 1], X, Y)
              & (A > 0))
    # barycentric weights of the projected point -> height of the crossing
    wa = (b2[:, 0] - X) * (c2[:, 1] - Y) - (b2[:, 1] - Y) * (c2[:, 0] - X)
    wb = (c2[:, 0] - X) * (a[:, 1] - Y) - (c2[:, 1] - Y) * (a[:, 0] - X)
    wc = (a[:, 0] - X) * (b2[:, 1] - Y) - (a[:, 1] - Y) * (b2[:, 0] - X)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = (wa * a[:, 2] + wb * b2[:, 2] + wc * c2[:, 2]) / A
    return [np.sort(z[j][inside[j]]) for j in range(x.shape[0])]


def _floor_div(a, b):
    return np.floor_divide(a, b)


def inside_sites(X: np.ndarray, tri: np.ndarray, dims, bc, origin=None, le_delta: float = 0.0) -> np.ndarray:
    """Boolean [nz, ny, nx]: the sites inside any cell.  X [C, nv, 3] holds
    positions (float64 arithmetic), or, with integer origins [C, 3], each
    cell's vertex offsets from its origin: then the crossings are found in
    those local coordinates in X's own precision, which lets a float32
    caller reproduce the decisions of a float32 implementation exactly.

    le_delta: with sheared periodic images (Sec. 2.5 reading: gradient axis
    z, flow axis x, image m displaced by m * le_delta along x) a node whose
    unwrapped z lies in image m = floor(z / nz) is inside when the cell's
    copy displaced by -m * le_delta contains it, i.e. its column is taken at
    cell-frame x + m * le_delta."""
    nx, ny, nz = dims
    n = (nx, ny, nz)
    mask = np.zeros((nz, ny, nx), dtype=bool)
    tri = np.asarray(tri, dtype=np.int64)
    X = np.asarray(X)
    dt = X.dtype.type if origin is not None else np.float64
    for c, V in enumerate(X.astype(dt)):
        o = np.zeros(3, np.int64) if origin is None else np.asarray(origin[c], dtype=np.int64)
        lo = np.ceil(V.min(axis=0)).astype(np.int64)
        hi = np.floor(V.max(axis=0)).astype(np.int64)
        images = [0] if le_delta == 0.0 else range(int(_floor_div(o[2] + lo[2], nz)),
                                                   int(_floor_div(o[2] + hi[2], nz)) + 1)
        for m in images:
            shift = dt(m) * dt(le_delta)
            xl = np.arange(np.ceil(V[:, 0].min() - shift), np.floor(V[:, 0].max() - shift) + 1).astype(np.int64)
            gx, gy = np.meshgrid(xl, np.arange(lo[1], hi[1] + 1), indexing="ij")
            gx, gy = gx.ravel(), gy.ravel()
            zs = crossings(V, tri, gx.astype(dt) + shift, gy.astype(dt))
            for ix, iy, z in zip(gx, gy, zs):
                for k in range(0, len(z) - 1, 2):
                    iz = np.arange(np.floor(z[k]) + 1, np.ceil(z[k + 1])).astype(np.int64) + o[2]
                    if le_delta != 0.0:
                        iz = iz[_floor_div(iz, nz) == m]   # the nodes of this image only
                    idx = [np.int64(ix) + o[0], np.int64(iy) + o[1], iz]
                    ok = np.ones(iz.shape, dtype=bool)
                    for d in range(3):
                        if bc[d] == WALL:
                            ok &= (idx[d] >= 0) & (idx[d] < n[d])
                        else:
                            idx[d] = np.mod(idx[d], n[d])
                    mask[idx[2][ok], np.broadcast_to(idx[1], iz.shape)[ok],
                         np.broadcast_to(idx[0], iz.shape)[ok]] = True
    return mask


def ratio_field(X: np.ndarray, tri: np.ndarray, dims, bc, ratios, origin=None,
                le_delta: float = 0.0) -> np.ndarray:
    """Viscosity ratio per site [nz, ny, nx] with one ratio per cell
    (mixtures of healthy and stiffened cells, Sec. 3.4): the ratio of the
    cell containing the site, the largest one where cells overlap, and 0
    where no cell does.  X, origin, le_delta: as for inside_sites."""
    nx, ny, nz = dims
    r = np.zeros((nz, ny, nx))
    for c in range(np.asarray(X).shape[0]):
        m = inside_sites(np.asarray(X)[c:c + 1], tri, dims, bc,
                         None if origin is None else np.asarray(origin)[c:c + 1], le_delta)
        r[m] = np.maximum(r[m], float(ratios[c]))
    return r


def tau_field(r: np.ndarray, tau: float) -> np.ndarray:
    """Per-site relaxation time from a ratio field (0: plasma)."""
    return np.where(r > 0, 0.5 + r * (tau - 0.5), tau)


def site_tau(mask: np.ndarray, tau: float, ratio: float) -> np.ndarray:
    """Per-site relaxation time: tau inside cells scaled to ratio times the viscosity."""
    return np.where(mask, 0.5 + ratio * (tau - 0.5), tau)
