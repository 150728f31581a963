"""Lees-Edwards sheared periodic images, float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.5 creates a boundary-free uniform shear: the domain is periodic in
every direction while two parallel boundaries carry opposing velocities,
and a cell crossing one of them re-enters on the other side.  The paper
does not spell out the scheme; the reading used here:
  * z is the gradient axis and x the flow axis; every axis is periodic;
  * the periodic image above the box (z + nz) is displaced by +Delta along
    x and moves with +U, the one below by -Delta and -U, where
    Delta(t) = U t mod nx at step t (t = 0 for the first step);
  * lattice: a population that reaches row z = 0 from below (or row
    z = nz - 1 from above) comes from the image's boundary row at the
    displaced position x - e_x + Delta (or x - e_x - Delta), which falls
    between nodes: all 19 post-collision populations of the two nodes
    around it are interpolated linearly along x, and the transferred
    population is changed by the Galilean term
    f_eq(rho~, u~ -/+ U) - f_eq(rho~, u~), rho~ and u~ the density and
    velocity of the interpolated set;
  * immersed boundary: a stencil node that lies in image m (m = floor of
    its unwrapped z index / nz) is reached through the vertex's image in
    that copy, at x - m Delta, so its x weights are those of X - m Delta;
    interpolation adds the image's velocity m U along x to the node's.
"""
from __future__ import annotations

import numpy as np

from . import ibm, lattice

E = lattice.E


def image_shift(u_le: float, t: int, nx: int) -> float:
    """Delta(t) = U t mod nx."""
    return float(np.mod(u_le * t, nx))


def _eq(rho, u):
    """Equilibrium of one set of populations: rho [...], u [3, ...] -> [19, ...]."""
    return lattice.equilibrium(rho, u)


def stream(post: np.ndarray, u_le: float, delta: float) -> np.ndarray:
    """Streaming of post-collision populations post [19, nz, ny, nx] with the
    sheared images: ordinary periodic streaming everywhere, except for the
    populations that cross the z boundary."""
    nz, ny, nx = post.shape[1:]
    out = np.empty_like(post)
    for i in range(19):
        out[i] = post[i]
        for d in range(3):
            if E[i, d] != 0:
                out[i] = np.roll(out[i], int(E[i, d]), axis=2 - d)
    xs = np.arange(nx, dtype=np.float64)
    for i in range(19):
        ez = int(E[i, 2])
        if ez == 0:
            continue
        # arriving at z = 0 from the image below (ez = +1) or at z = nz - 1
        # from the image above (ez = -1)
        dst_z, src_z, sign = (0, nz - 1, -1.0) if ez > 0 else (nz - 1, 0, +1.0)
        pos = xs - E[i, 0] - sign * delta          # displaced source x along the image row
        x0 = np.floor(pos)
        s = pos - x0
        x0 = x0.astype(np.int64) % nx
        x1 = (x0 + 1) % nx
        row = np.roll(post[:, src_z], int(E[i, 1]), axis=1)    # y - e_y
        h = (1.0 - s) * row[:, :, x0] + s * row[:, :, x1]       # [19, ny, nx]
        rho = h.sum(axis=0)
        u = np.tensordot(E.T.astype(np.float64), h, axes=(1, 0)) / rho
        v = u.copy()
        v[0] += sign * u_le
        out[i, dst_z] = h[i] + _eq(rho, v)[i] - _eq(rho, u)[i]
    return out


def _x_of_image(X, m, delta):
    """x coordinate of a vertex as seen from image m."""
    return X[:, 0] - m * delta


def spread(X: np.ndarray, Fv: np.ndarray, dims, delta: float, kernel: int = 4) -> np.ndarray:
    """Force density of vertex forces on the sheared-periodic lattice."""
    phi, ks = ibm._stencil(kernel)
    nx, ny, nz = dims
    out = np.zeros((3, nz * ny * nx))
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    Fv = np.asarray(Fv, dtype=np.float64).reshape(-1, 3)
    for kz in ks:
        zn = np.floor(X[:, 2]).astype(np.int64) + kz
        m = np.floor_divide(zn, nz)
        iz = np.mod(zn, nz)
        wz = phi(X[:, 2] - zn)
        xe = _x_of_image(X, m, delta)
        for ky in ks:
            yn = np.floor(X[:, 1]).astype(np.int64) + ky
            iy = np.mod(yn, ny)
            wy = phi(X[:, 1] - yn)
            for kx in ks:
                xn = np.floor(xe).astype(np.int64) + kx
                ix = np.mod(xn, nx)
                w = phi(xe - xn) * wy * wz
                s = (iz * ny + iy) * nx + ix
                for d in range(3):
                    out[d] += np.bincount(s, weights=w * Fv[:, d], minlength=out.shape[1])
    return out.reshape(3, nz, ny, nx)


def interpolate(u: np.ndarray, X: np.ndarray, dims, u_le: float, delta: float,
                kernel: int = 4) -> np.ndarray:
    """Vertex velocity on the sheared-periodic lattice: a node in image m
    carries its velocity plus m U along x."""
    phi, ks = ibm._stencil(kernel)
    nx, ny, nz = dims
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    uf = u.reshape(3, -1)
    U = np.zeros_like(X)
    for kz in ks:
        zn = np.floor(X[:, 2]).astype(np.int64) + kz
        m = np.floor_divide(zn, nz)
        iz = np.mod(zn, nz)
        wz = phi(X[:, 2] - zn)
        xe = _x_of_image(X, m, delta)
        for ky in ks:
            yn = np.floor(X[:, 1]).astype(np.int64) + ky
            iy = np.mod(yn, ny)
            wy = phi(X[:, 1] - yn)
            for kx in ks:
                xn = np.floor(xe).astype(np.int64) + kx
                ix = np.mod(xn, nx)
                w = phi(xe - xn) * wy * wz
                s = (iz * ny + iy) * nx + ix
                val = uf[:, s].T.copy()
                val[:, 0] += m * u_le
                U += w[:, None] * val
    return U
