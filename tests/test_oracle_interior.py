"""Pins of the interior-site oracle (ray parity) and of per-site relaxation.

* sphere: sites well inside the inscribed sphere of an icosphere mesh are
  inside, sites outside its circumscribed sphere are outside;
* the parity does not depend on the ray direction: casting along x instead
  of z (coordinates permuted) marks the same sites for a generic placement;
* translating a cell across a periodic boundary by whole nodes translates
  its mask;
* per-site relaxation is local: with one relaxation time everywhere it is
  the scalar collision, and each site relaxes with its own time.
"""
import numpy as np

from oracle import interior, lattice
from workloads import rbc_mesh
from workloads.mesh import sphere_mesh


def test_sphere_inside_outside():
    R = 7.0
    V, tri = sphere_mesh(3, R)
    c = np.array([12.31, 11.77, 10.52])
    mask = interior.inside_sites((V + c)[None], tri, (24, 24, 22), (0, 0, 0))
    z, y, x = np.meshgrid(np.arange(22), np.arange(24), np.arange(24), indexing="ij")
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    r_in = R * 0.99     # faces of a level-3 icosphere lie within 1% of R
    assert mask[r < r_in - 1e-6].all()
    assert not mask[r > R + 1e-6].any()


def test_parity_independent_of_ray_direction():
    rest, tri = rbc_mesh()
    rng = np.random.default_rng(5)
    th = rng.uniform(0, 2 * np.pi)
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    Ry = np.array([[np.cos(0.7), 0, np.sin(0.7)], [0, 1.0, 0], [-np.sin(0.7), 0, np.cos(0.7)]])
    X = rest @ (Rz @ Ry).T + np.array([16.137, 15.791, 14.263])
    dims = (32, 32, 30)
    mz = interior.inside_sites(X[None], tri, dims, (0, 0, 0))
    # cast along x: swap the x and z coordinates (orientation flips, parity does not)
    Xs = X[:, [2, 1, 0]]
    mx = interior.inside_sites(Xs[None], tri, (dims[2], dims[1], dims[0]), (0, 0, 0))
    assert mz.sum() > 500
    assert np.array_equal(mz, np.transpose(mx, (2, 1, 0)))


def test_periodic_translation():
    rest, tri = rbc_mesh()
    X = rest + np.array([10.21, 9.87, 8.43])
    dims = (20, 20, 18)
    m0 = interior.inside_sites(X[None], tri, dims, (0, 0, 0))
    shift = np.array([13, -7, 11])
    m1 = interior.inside_sites((X + shift)[None], tri, dims, (0, 0, 0))
    assert np.array_equal(np.roll(m0, (shift[2], shift[1], shift[0]), axis=(0, 1, 2)), m1)


def test_per_site_relaxation_is_local():
    rng = np.random.default_rng(6)
    f = lattice.init_equilibrium((6, 5, 4)) + 1e-3 * rng.standard_normal((19, 6, 5, 4))
    F = 1e-5 * rng.standard_normal((3, 6, 5, 4))
    rho, u = lattice.moments(f, F)
    ref = lattice.collide(f, rho, u, F, 0.8)
    assert np.allclose(lattice.collide(f, rho, u, F, np.full((6, 5, 4), 0.8)), ref, rtol=0, atol=1e-16)
    tau = np.where(rng.uniform(size=(6, 5, 4)) < 0.5, 0.8, 2.5)
    post = lattice.collide(f, rho, u, F, tau)
    ref2 = lattice.collide(f, rho, u, F, 2.5)
    sel = tau == 2.5
    assert np.allclose(post[:, sel], ref2[:, sel], rtol=0, atol=1e-16)
    assert np.allclose(post[:, ~sel], ref[:, ~sel], rtol=0, atol=1e-16)


def test_local_float32_mode_matches_positions():
    """Offsets from integer origins in float32 mark what the float64
    positions mark (generic placements: no crossing within rounding of a
    node), including cells that wrap across periodic sides."""
    rest, tri = rbc_mesh()
    rng = np.random.default_rng(8)
    dims = (40, 36, 34)
    origin = np.array([[3, 30, 5], [20, 17, 30], [37, 2, 17]])
    off = np.stack([rest @ np.linalg.qr(rng.standard_normal((3, 3)))[0].T + rng.uniform(0, 1, 3)
                    for _ in range(3)])
    off32 = off.astype(np.float32)
    X = origin[:, None, :] + off32.astype(np.float64)
    m64 = interior.inside_sites(X, tri, dims, (0, 0, 0))
    m32 = interior.inside_sites(off32, tri, dims, (0, 0, 0), origin=origin)
    assert m64.sum() > 1500
    assert np.array_equal(m64, m32)


def test_ratio_field_per_cell():
    """One ratio per cell: uniform ratios reproduce the single-ratio form;
    disjoint cells keep their own ratio; overlaps take the largest, in any
    cell order."""
    rest, tri = rbc_mesh()
    dims = (40, 24, 22)
    A = rest + np.array([10.3, 11.6, 10.9])
    B = rest + np.array([29.7, 12.2, 11.3])          # disjoint from A
    Cc = rest + np.array([14.1, 12.4, 11.1])         # overlaps A
    X = np.stack([A, B])
    r = interior.ratio_field(X, tri, dims, (0, 0, 0), [5.0, 5.0])
    assert np.array_equal(interior.tau_field(r, 0.9),
                          interior.site_tau(interior.inside_sites(X, tri, dims, (0, 0, 0)), 0.9, 5.0))
    r = interior.ratio_field(X, tri, dims, (0, 0, 0), [5.0, 2.0])
    mA = interior.inside_sites(A[None], tri, dims, (0, 0, 0))
    mB = interior.inside_sites(B[None], tri, dims, (0, 0, 0))
    assert mA.sum() > 300 and mB.sum() > 300 and not (mA & mB).any()
    assert (r[mA] == 5.0).all() and (r[mB] == 2.0).all() and (r[~(mA | mB)] == 0).all()
    mC = interior.inside_sites(Cc[None], tri, dims, (0, 0, 0))
    both = mA & mC
    assert both.sum() > 50
    r1 = interior.ratio_field(np.stack([A, Cc]), tri, dims, (0, 0, 0), [0.5, 3.0])
    r2 = interior.ratio_field(np.stack([Cc, A]), tri, dims, (0, 0, 0), [3.0, 0.5])
    assert np.array_equal(r1, r2)
    assert (r1[both] == 3.0).all() and (r1[mA & ~mC] == 0.5).all()


def test_per_site_relaxation_conserves_mass_and_momentum():
    """BGK with a per-site relaxation time keeps the collision invariants:
    mass unchanged, momentum changed by exactly the Guo force (Sec. 2.3)."""
    rng = np.random.default_rng(9)
    shape = (6, 5, 4)
    f = lattice.init_equilibrium(shape) + 1e-3 * rng.standard_normal((19,) + shape)
    F = 1e-5 * rng.standard_normal((3,) + shape)
    rho, u = lattice.moments(f, F)
    tau = 0.5 + rng.uniform(0.05, 4.0, shape)
    post = lattice.collide(f, rho, u, F, tau)
    e = np.array(lattice.E, dtype=np.float64)
    assert np.allclose(post.sum(axis=0), f.sum(axis=0), rtol=0, atol=1e-15)
    mom = lambda g: np.einsum("qd,q...->d...", e, g)
    assert np.allclose(mom(post) - mom(f), F, rtol=0, atol=1e-15)


def test_sheared_images_marks():
    """Lees-Edwards images (Sec. 2.5 reading): with no shift the marks are the
    periodic ones; with an integer shift D the nodes that lie in the image
    above (z wrapped from nz) are the periodic marks moved by -D along x,
    and the nodes of the cell's own image are unchanged; float32 local
    decisions agree with float64 positions for a fractional shift."""
    rest, tri = rbc_mesh()
    dims = (40, 28, 24)
    X = (rest @ np.linalg.qr(np.random.default_rng(10).standard_normal((3, 3)))[0].T
         + np.array([19.37, 13.81, 22.64]))[None]     # straddles z = nz
    m0 = interior.inside_sites(X, tri, dims, (0, 0, 0))
    assert np.array_equal(interior.inside_sites(X, tri, dims, (0, 0, 0), le_delta=0.0), m0)
    D = 7
    mD = interior.inside_sites(X, tri, dims, (0, 0, 0), le_delta=float(D))
    zu = np.arange(int(np.ceil(X[0, :, 2].min())), int(np.floor(X[0, :, 2].max())) + 1)
    above = np.unique(np.mod(zu[zu >= dims[2]], dims[2]))
    below = np.unique(zu[zu < dims[2]])
    assert above.size > 0 and below.size > 0 and not np.intersect1d(above, below).size
    assert m0[above].sum() > 100
    assert np.array_equal(mD[above], np.roll(m0[above], -D, axis=2))
    assert np.array_equal(mD[below], m0[below])
    # fractional shift: float32 local decisions equal float64 positions
    origin = np.floor(X[0].mean(axis=0)).astype(np.int64)[None]
    off32 = (X - origin[:, None, :]).astype(np.float32)
    X64 = origin[:, None, :] + off32.astype(np.float64)
    d = 5.37
    assert np.array_equal(interior.inside_sites(off32, tri, dims, (0, 0, 0), origin=origin, le_delta=d),
                          interior.inside_sites(X64, tri, dims, (0, 0, 0), le_delta=d))
