"""Pins of the binning oracle (brute force) and of the coupled step oracle.

Binning: every list is re-derived by enumerating all lattice nodes of every
tile.  Coupled step (Sec. 2.3 explicit IBM coupling, Sec. 2.6 Euler
integration): an undeformed cell in uniform flow translates rigidly by the
flow velocity per step, the total momentum of a force-free periodic
suspension is conserved, and mass is conserved.
"""
import numpy as np
import pytest

from oracle import binning, lattice, step
from workloads import jitter_cells, rbc_mesh, tiny_periodic
from workloads.configs import Lattice, place_cells, random_rotation, K_REF


def _brute_bins(origin, off, dims, bc):
    T = [(n + 7) // 8 for n in dims]
    C, V = off.shape[:2]
    owner = np.zeros((C, V), dtype=np.int64)
    for c in range(C):
        for v in range(V):
            p = []
            for d in range(3):
                q = int(origin[c, d]) + int(np.floor(np.float32(off[c, v, d])))
                q = min(max(q, 0), dims[d] - 1) if bc[d] == 1 else q % dims[d]
                p.append(q)
            owner[c, v] = ((p[2] // 8) * T[1] + p[1] // 8) * T[0] + p[0] // 8
    cover = []
    for c in range(C):
        rng_nodes = []
        for d in range(3):
            lo = int(origin[c, d]) + int(np.floor(off[c, :, d].min())) - 1
            hi = int(origin[c, d]) + int(np.floor(off[c, :, d].max())) + 2
            nodes = set()
            for q in range(lo, hi + 1):
                nodes.add(min(max(q, 0), dims[d] - 1) if bc[d] == 1 else q % dims[d])
            rng_nodes.append(nodes)
        tiles = set()
        for tz in range(T[2]):
            for ty in range(T[1]):
                for tx in range(T[0]):
                    xs = range(tx * 8, min(tx * 8 + 8, dims[0]))
                    ys = range(ty * 8, min(ty * 8 + 8, dims[1]))
                    zs = range(tz * 8, min(tz * 8 + 8, dims[2]))
                    if (any(x in rng_nodes[0] for x in xs) and any(y in rng_nodes[1] for y in ys)
                            and any(z in rng_nodes[2] for z in zs)):
                        tiles.add((tz * T[1] + ty) * T[0] + tx)
        cover.append(tiles)
    return owner, cover


@pytest.mark.parametrize("dims,bc", [((16, 16, 16), (0, 0, 0)), ((20, 17, 24), (0, 1, 0))])
def test_binning_brute_force(dims, bc):
    rng = np.random.default_rng(7)
    rest64, _ = rbc_mesh()
    C = 3
    cen = rng.uniform(0, 1, (C, 3)) * np.array(dims)
    if bc[1] == 1:
        cen[:, 1] = dims[1] / 2
    cells = place_cells(0.5 * rest64, cen, np.stack([random_rotation(rng) for _ in range(C)]),
                        np.repeat(K_REF[None], C, 0))
    owner, vptr, tverts, cptr, tcells = binning.bins(cells.origin, cells.offsets, dims, bc)
    bo, cover = _brute_bins(cells.origin, cells.offsets, dims, bc)
    assert (owner == bo.ravel()).all()
    nt = len(vptr) - 1
    for t in range(nt):
        vs = tverts[vptr[t]:vptr[t + 1]]
        assert list(vs) == sorted(np.nonzero(bo.ravel() == t)[0])
        cs = tcells[cptr[t]:cptr[t + 1]]
        assert list(cs) == [c for c in range(C) if t in cover[c]]


def test_uniform_flow_translates_rest_cell():
    lat = Lattice(24, 24, 24)
    rest64, tri = rbc_mesh()
    m = step.make_model(lat, rest64, tri, K_REF[None])
    u0 = np.array([0.013, -0.007, 0.004])
    u = np.broadcast_to(u0[:, None, None, None], (3, 24, 24, 24))
    f = lattice.equilibrium(np.ones((24, 24, 24)), u)
    X = rest64[None] + np.array([11.3, 12.1, 10.7])
    f1, X1, info = step.step(m, f, X)
    assert np.abs(info["Fv"]).max() < 1e-17
    assert np.abs(X1 - X - u0).max() < 1e-14          # rounding of X ~ 20
    _, u1 = lattice.moments(f1)
    assert np.abs(u1 - u0[:, None, None, None]).max() < 1e-15


def test_coupled_momentum_and_mass_conservation():
    """Force-free periodic suspension: internal membrane forces sum to zero,
    so fluid momentum and mass are conserved by the coupled step."""
    w = tiny_periodic(seed=11, n=(20, 18, 22), n_cells=2)
    rng = np.random.default_rng(0)
    cells = jitter_cells(rng, w.cells, 0.05)
    m = step.make_model(w.lattice, w.rest_pos, w.tri, cells.k, traction=None)
    f = lattice.unshift(np.zeros((19,) + w.lattice.shape)) + 1e-4 * rng.standard_normal((19,) + w.lattice.shape)
    X = cells.positions64()
    E = lattice.E.T.astype(float)
    p0 = np.tensordot(E, f, 1).sum(axis=(1, 2, 3))
    m0 = f.sum()
    for _ in range(3):
        f, X, info = step.step(m, f, X)
        assert np.abs(info["Fv"]).max() > 1e-6
    p1 = np.tensordot(E, f, 1).sum(axis=(1, 2, 3))
    assert np.abs(p1 - p0).max() < 1e-13
    assert abs(f.sum() - m0) < 1e-10


def test_sheared_touch_lists_special_cases():
    # Lees-Edwards touch lists: no shift, and a shift of whole periods, are
    # the plain periodic lists; a shift of one tile moves the x tiles of the
    # nodes beyond the top z boundary by one tile (worked by hand)
    rng = np.random.default_rng(3)
    dims = (32, 24, 40)
    o = rng.integers(0, 40, (3, 3))
    off = rng.uniform(-8.0, 8.0, (3, 30, 3)).astype(np.float32)
    plain = binning.touch_lists(o, off, dims, (0, 0, 0), 4)
    for delta in (0.0, 32.0, 64.0):
        got = binning.touch_lists(o, off, dims, (0, 0, 0), 4, le_delta=delta)
        assert np.array_equal(got[0], plain[0]) and np.array_equal(got[1], plain[1]), delta
    # one vertex at x = 12.5, y = 4.5, z = 39.5: z nodes 38, 39 (image 0:
    # tile 4) and 40, 41 (image 1: wrapped 0, 1, tile 0, x displaced by -8)
    o1 = np.zeros((1, 3), dtype=np.int64)
    off1 = np.array([[[12.5, 4.5, 39.5]]], dtype=np.float32)
    ptr, vid = binning.touch_lists(o1, off1, dims, (0, 0, 0), 4, le_delta=8.0)
    T = binning.tiles_per_axis(dims)
    tiles = {t for t in range(T[0] * T[1] * T[2]) if ptr[t + 1] > ptr[t]}
    # x nodes 11..14 (tile 1) in image 0, 3..6 (tile 0) in image 1; y nodes 3..6 (tile 0)
    expect = {(4 * T[1] + 0) * T[0] + 1, (0 * T[1] + 0) * T[0] + 0}
    assert tiles == expect


def _brute_touch(origin, off, dims, bc, kernel):
    """(tile, vertex) pairs by enumeration: for every tile, every node in it,
    and for every vertex the nodes of its stencil (walls drop the nodes past
    them): the vertex is listed for the tile when one of its stencil nodes is
    one of the tile's nodes."""
    K = kernel
    T = [(n + 7) // 8 for n in dims]
    off = np.asarray(off, dtype=np.float32)
    C, V = off.shape[:2]
    first = -1 if K == 4 else 0
    base = (origin[:, None, :].astype(np.int64) + np.floor(off).astype(np.int64) + first).reshape(-1, 3)
    # stencil node sets, one boolean row per vertex and per axis over the nodes of that axis
    reach = []
    for d in range(3):
        n = dims[d]
        hit = np.zeros((C * V, n), dtype=bool)
        for k in range(K):
            p = base[:, d] + k
            if bc[d] == 1:
                ok = (p >= 0) & (p < n)
                hit[np.nonzero(ok)[0], p[ok]] = True
            else:
                hit[np.arange(C * V), np.mod(p, n)] = True
        reach.append(hit)
    out = {}
    for tz in range(T[2]):
        for ty in range(T[1]):
            for tx in range(T[0]):
                t = (tz * T[1] + ty) * T[0] + tx
                xs = np.arange(tx * 8, min(tx * 8 + 8, dims[0]))
                ys = np.arange(ty * 8, min(ty * 8 + 8, dims[1]))
                zs = np.arange(tz * 8, min(tz * 8 + 8, dims[2]))
                # every node (x, y, z) of the tile against every vertex
                node_hit = (reach[0][:, xs][:, None, None, :] & reach[1][:, ys][:, None, :, None]
                            & reach[2][:, zs][:, :, None, None])
                out[t] = np.nonzero(node_hit.reshape(C * V, -1).any(axis=1))[0]
    return out


@pytest.mark.parametrize("kernel", [4, 2])
@pytest.mark.parametrize("dims,bc", [
    ((16, 16, 16), (0, 0, 0)),
    ((33, 20, 25), (0, 1, 0)),     # ragged tiles, y walls
    ((17, 18, 26), (0, 0, 0)),     # last tiles 1-2 nodes wide: a stencil meets 3 tiles
    ((6, 20, 5), (0, 0, 0)),       # sides below 8
    ((6, 20, 5), (0, 0, 1)),       # sides below 8, a wall on the 5-node axis
    ((25, 19, 18), (1, 0, 0)),     # x walls, ragged
])
def test_touch_lists_brute_force(dims, bc, kernel):
    rng = np.random.default_rng(sum(dims) + kernel)
    rest64, _ = rbc_mesh()
    C = 3
    cen = rng.uniform(0, 1, (C, 3)) * np.array(dims)
    for d in range(3):
        if bc[d] == 1:   # keep the cells inside the walls, near them
            cen[:, d] = np.array([2.5, dims[d] / 2, dims[d] - 3.0])
    cen[0, 0] = dims[0] - 0.7 if bc[0] == 0 else cen[0, 0]   # straddle the periodic x boundary
    cells = place_cells(0.35 * rest64, cen, np.stack([random_rotation(rng) for _ in range(C)]),
                        np.repeat(K_REF[None], C, 0))
    off = cells.offsets.copy()
    # some vertices exactly on nodes and just below them
    off[1, :40] = np.round(off[1, :40])
    off[2, :40] = np.nextafter(np.round(off[2, :40]), np.float32(-np.inf))
    ptr, vid = binning.touch_lists(cells.origin, off, dims, bc, kernel)
    want = _brute_touch(cells.origin, off, dims, bc, kernel)
    nt = len(ptr) - 1
    assert nt == len(want)
    total = 0
    for t in range(nt):
        got = vid[ptr[t]:ptr[t + 1]]
        assert np.array_equal(got, want[t]), t
        total += len(got)
    assert total > C * off.shape[1] // 2
