"""Immersed-boundary spreading and interpolation, float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.3 couples the Lagrangian membrane vertices to the Eulerian lattice
with Peskin's immersed-boundary method: vertex forces enter the fluid as an
external force field, and the fluid velocity is interpolated back to the
vertices.  Readings:
  * kernel: Peskin's 4-point function phi4 (default) on the nodes
    floor(X)-1 .. floor(X)+2 per axis; the linear hat (the paper's "linear
    interpolation") is kept as the 2-point option on floor(X), floor(X)+1;
  * the 3-D weight is the product of the per-axis weights;
  * periodic axes wrap; on a wall axis, nodes beyond the wall receive no
    force and contribute the velocity of the wall on that side.
Lattice node index i sits at coordinate x = i.
"""
from __future__ import annotations

import numpy as np

WALL = 1


def _abs(r):
    """|r| for real arrays; for complex ones (the complex-step gradient) the
    sign is decided by the real part, which continues |r| analytically."""
    r = np.asarray(r)
    r = r if np.iscomplexobj(r) else r.astype(np.float64)
    return np.where(r.real < 0.0, -r, r)


def phi4(r):
    """Peskin's 4-point regularised delta function (Peskin 2002)."""
    r = _abs(r)
    out = np.zeros_like(r)
    a = r.real <= 1.0
    b = (r.real > 1.0) & (r.real < 2.0)
    out[a] = (3.0 - 2.0 * r[a] + np.sqrt(1.0 + 4.0 * r[a] - 4.0 * r[a] ** 2)) / 8.0
    out[b] = (5.0 - 2.0 * r[b] - np.sqrt(-7.0 + 12.0 * r[b] - 4.0 * r[b] ** 2)) / 8.0
    return out


def phi2(r):
    """Linear hat max(0, 1 - |r|)."""
    r = _abs(r)
    return np.where(r.real < 1.0, 1.0 - r, 0.0)


def _array(a):
    """float64 array, or complex128 for the complex-step gradient."""
    a = np.asarray(a)
    return a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)


def _scatter_add(idx, val, n):
    """Sums of val over equal idx, length n (real and imaginary parts apart)."""
    if np.iscomplexobj(val):
        return np.bincount(idx, weights=val.real, minlength=n) + 1j * np.bincount(idx, weights=val.imag, minlength=n)
    return np.bincount(idx, weights=val, minlength=n)


def _stencil(kernel: int):
    if kernel == 4:
        return phi4, (-1, 0, 1, 2)
    if kernel == 2:
        return phi2, (0, 1)
    raise ValueError("kernel must be 4 or 2")


def _axis_nodes(x, k, n, bc):
    """Node index along one axis for offset k, and whether it is inside the fluid."""
    node = np.floor(np.real(x)).astype(np.int64) + k
    if bc == WALL:
        inside = (node >= 0) & (node < n)
        return node, inside
    return np.mod(node, n), np.ones(node.shape, dtype=bool)


def spread(X: np.ndarray, Fv: np.ndarray, dims, bc, kernel: int = 4) -> np.ndarray:
    """Eulerian force density F(x) = sum_v F_v phi(X_v,x - x) phi(..y..) phi(..z..).

    X, Fv: [M,3] float64.  dims = (nx, ny, nz).  Returns [3, nz, ny, nx].
    """
    phi, ks = _stencil(kernel)
    nx, ny, nz = dims
    X = _array(X).reshape(-1, 3)
    Fv = _array(Fv).reshape(-1, 3)
    out = np.zeros((3, nz * ny * nx), dtype=np.result_type(X, Fv))
    for kz in ks:
        iz, okz = _axis_nodes(X[:, 2], kz, nz, bc[2])
        wz = phi(X[:, 2] - (np.floor(X[:, 2].real) + kz))
        for ky in ks:
            iy, oky = _axis_nodes(X[:, 1], ky, ny, bc[1])
            wy = phi(X[:, 1] - (np.floor(X[:, 1].real) + ky))
            for kx in ks:
                ix, okx = _axis_nodes(X[:, 0], kx, nx, bc[0])
                wx = phi(X[:, 0] - (np.floor(X[:, 0].real) + kx))
                ok = okx & oky & okz
                w = (wx * wy * wz)[ok]
                s = ((iz * ny + iy) * nx + ix)[ok]
                for d in range(3):
                    out[d] += _scatter_add(s, w * Fv[ok, d], out.shape[1])
    return out.reshape(3, nz, ny, nx)


def interpolate(u: np.ndarray, X: np.ndarray, dims, bc, wall_u_lo, wall_u_hi,
                kernel: int = 4) -> np.ndarray:
    """Vertex velocity U_v = sum_x u(x) phi phi phi over the same stencil.

    u: [3, nz, ny, nx].  Nodes past a wall contribute that wall's velocity.
    Returns [M,3].
    """
    phi, ks = _stencil(kernel)
    nx, ny, nz = dims
    n = (nx, ny, nz)
    X = _array(X).reshape(-1, 3)
    uf = u.reshape(3, -1)
    lo = np.asarray(wall_u_lo, dtype=np.float64)
    hi = np.asarray(wall_u_hi, dtype=np.float64)
    U = np.zeros(X.shape, dtype=np.result_type(X, uf))
    for kz in ks:
        for ky in ks:
            for kx in ks:
                kk = (kx, ky, kz)
                w = np.ones(X.shape[0])
                idx = []
                inside = np.ones(X.shape[0], dtype=bool)
                below = np.zeros(X.shape[0], dtype=bool)
                above = np.zeros(X.shape[0], dtype=bool)
                for d in range(3):
                    node = np.floor(X[:, d].real).astype(np.int64) + kk[d]
                    w = w * phi(X[:, d] - node)
                    if bc[d] == WALL:
                        below |= node < 0
                        above |= node >= n[d]
                        inside &= (node >= 0) & (node < n[d])
                        idx.append(np.clip(node, 0, n[d] - 1))
                    else:
                        idx.append(np.mod(node, n[d]))
                s = (idx[2] * ny + idx[1]) * nx + idx[0]
                val = uf[:, s].T.copy()
                val[below] = lo
                val[above] = hi
                U += w[:, None] * val
    return U
