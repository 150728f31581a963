"""Cell and vertex binning to lattice tiles (integer work, oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

The paper distributes lattice and cells over processors by domain
decomposition and tracks which region owns which cell (Sec. 2.6).  On one
device the same bookkeeping becomes binning to cubic lattice tiles of side
8.  Reading of the rules (exact on the float32 positions the device holds):
  * vertex owner: node p_d = origin_d + floor(offset_d), wrapped into
    [0, N_d) on every axis (a walled axis clamps), tile coordinate
    p_d >> 3, tile id (tz * Ty + ty) * Tx + tx with T_d = ceil(N_d / 8);
  * cell coverage: per axis the node range
    [origin + floor(min offset) - 1, origin + floor(max offset) + 2]
    (the 4-point stencil reach), wrapped on periodic axes and clamped on
    walled ones; the cell covers every tile the range meets;
  * touch lists: per tile the vertices whose IBM stencil nodes
    (floor(X)-1 .. floor(X)+2 for the 4-point kernel, floor(X) ..
    floor(X)+1 for the 2-point one; walls drop outside nodes) lie in it;
  * CSR lists sorted by (tile, cell) and (tile, cell, vertex).
  * with Lees-Edwards images (Sec. 2.5 reading; periodic axes, shift Delta
    along x per image across z): a z stencil node p lies in image
    m = floor(p / N_z), and its x nodes are those of the vertex displaced
    to x - m Delta.  The displaced coordinate decides integer tiles, so it
    is taken as the device takes it: offset - m Delta in float32 with one
    rounding (a fused multiply-add).
"""
from __future__ import annotations

import numpy as np

WALL = 1
TILE = 8


def tiles_per_axis(dims):
    return tuple((n + TILE - 1) // TILE for n in dims)


def _wrap(p, n, bc):
    if bc == WALL:
        return np.clip(p, 0, n - 1)
    return np.mod(p, n)


def vertex_owner(origin, offsets, dims, bc):
    """Owner tile id of every vertex, int64 [C, V]."""
    off = np.asarray(offsets, dtype=np.float32)
    T = tiles_per_axis(dims)
    t = []
    for d in range(3):
        p = origin[:, None, d].astype(np.int64) + np.floor(off[:, :, d]).astype(np.int64)
        t.append(_wrap(p, dims[d], bc[d]) // TILE)
    return (t[2] * T[1] + t[1]) * T[0] + t[0]


def cell_tiles(origin, offsets, dims, bc, c):
    """Sorted tile ids covered by cell c."""
    off = np.asarray(offsets[c], dtype=np.float32)
    T = tiles_per_axis(dims)
    per_axis = []
    for d in range(3):
        lo = int(origin[c, d]) + int(np.floor(off[:, d].min())) - 1
        hi = int(origin[c, d]) + int(np.floor(off[:, d].max())) + 2
        nodes = _wrap(np.arange(lo, hi + 1), dims[d], bc[d])
        per_axis.append(np.unique(nodes // TILE))
    tz, ty, tx = np.meshgrid(per_axis[2], per_axis[1], per_axis[0], indexing="ij")
    return np.unique(((tz * T[1] + ty) * T[0] + tx).ravel())


def bins(origin, offsets, dims, bc):
    """CSR binning: (owner [C*V], vert_ptr [NT+1], tile_vertices, cell_ptr [NT+1], tile_cells)."""
    C, V = offsets.shape[0], offsets.shape[1]
    T = tiles_per_axis(dims)
    nt = T[0] * T[1] * T[2]
    owner = vertex_owner(origin, offsets, dims, bc).ravel()
    gidx = np.arange(C * V)
    order = np.lexsort((gidx, owner))
    vert_ptr = np.zeros(nt + 1, dtype=np.int64)
    np.add.at(vert_ptr, owner + 1, 1)
    vert_ptr = np.cumsum(vert_ptr)
    pairs = []
    for c in range(C):
        for t in cell_tiles(origin, offsets, dims, bc, c):
            pairs.append((int(t), c))
    pairs = np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)
    cell_ptr = np.zeros(nt + 1, dtype=np.int64)
    np.add.at(cell_ptr, pairs[:, 0] + 1, 1)
    cell_ptr = np.cumsum(cell_ptr)
    return owner, vert_ptr, gidx[order], cell_ptr, pairs[:, 1]


def _sheared_x(off_x, m, delta):
    """float32(off_x - m * delta) rounded once, as a fused multiply-add:
    the product of a small integer and a float32 and the difference are
    exact in float64, so one rounding to float32 follows."""
    return np.float32(np.float64(np.float32(off_x)) - np.float64(m) * np.float64(np.float32(delta)))


def touch_lists(origin, offsets, dims, bc, kernel=4, le_delta=None):
    """CSR (ptr [NT+1], vertex ids) of the tiles each vertex's stencil
    reaches; le_delta: the image shift with Lees-Edwards images (None: no
    images)."""
    off = np.asarray(offsets, dtype=np.float32)
    C, V = off.shape[:2]
    T = tiles_per_axis(dims)
    ks = (-1, 0, 1, 2) if kernel == 4 else (0, 1)
    pairs = set()
    for c in range(C):
        for v in range(V):
            if le_delta is not None:   # node by node: x depends on the z node's image
                yb = int(origin[c, 1]) + int(np.floor(off[c, v, 1]))
                zb = int(origin[c, 2]) + int(np.floor(off[c, v, 2]))
                for kz in ks:
                    p = zb + kz
                    m = p // dims[2]
                    xm = _sheared_x(off[c, v, 0], m, le_delta)
                    xb = int(origin[c, 0]) + int(np.floor(xm))
                    for ky in ks:
                        for kx in ks:
                            t = (((p % dims[2]) // TILE) * T[1] + ((yb + ky) % dims[1]) // TILE) * T[0] \
                                + ((xb + kx) % dims[0]) // TILE
                            pairs.add((t, c * V + v))
                continue
            axes = []
            for d in range(3):
                base = int(origin[c, d]) + int(np.floor(off[c, v, d]))
                tiles = set()
                for k in ks:
                    p = base + k
                    if bc[d] == WALL and not (0 <= p < dims[d]):
                        continue
                    tiles.add((p % dims[d]) // TILE)
                axes.append(tiles)
            for tz in axes[2]:
                for ty in axes[1]:
                    for tx in axes[0]:
                        pairs.add(((tz * T[1] + ty) * T[0] + tx, c * V + v))
    pairs = np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)
    nt = T[0] * T[1] * T[2]
    ptr = np.zeros(nt + 1, dtype=np.int64)
    np.add.at(ptr, pairs[:, 0] + 1, 1)
    return np.cumsum(ptr), pairs[:, 1]
