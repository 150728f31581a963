"""Interior viscosity on the device against the oracle.

Sites inside the cells (ray parity along z) relax with tau_in = 1/2 +
ratio (tau - 1/2) (Sec. 1, Sec. 3.4 reading, oracle/interior.py).  Bars:
the inside marks are integer work decided in float32 from the cells'
offsets: bit-exact against the oracle's float32 local-coordinate mode,
before and after the cells have moved on the device (the device's own
float32 positions are the defined input of that marking).  Coupled steps
with ratio 5: populations within 1e-4 after 12 steps (1e-5 per step
accumulated) and positions within that fraction of the displacement plus
the rounding of the float32 offsets, against the FP64 oracle.
"""
import numpy as np
import pytest

from oracle import interior, lattice, step
from workloads import jitter_cells, random_shifted_populations, rbc_mesh, tiny_periodic
from workloads.configs import Lattice, place_cells, random_rotation

from gpu_common import make_sim, oracle_model, oracle_state, relerr

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _oracle_mask(sim, lat, tri):
    o, off, _ = sim.read_vertices()
    return interior.inside_sites(off, tri, (lat.nx, lat.ny, lat.nz), lat.bc, origin=o)


@pytest.mark.parametrize("walls", [-1, 2, 0])
def test_marks_match_oracle(walls):
    w = tiny_periodic(seed=41 + walls, n=(32, 28, 24), n_cells=3, walls=walls)
    cells = jitter_cells(np.random.default_rng(42), w.cells, 0.05)
    sim = make_sim(w, cells)
    sim.init_equilibrium()
    sim.set_interior_viscosity(5.0)
    dev = sim.read_interior()
    ref = interior.inside_sites(cells.offsets, w.tri, (w.lattice.nx, w.lattice.ny, w.lattice.nz),
                                w.lattice.bc, origin=cells.origin)
    print("walls", walls, "inside", int(ref.sum()), "mismatch", int((dev.astype(bool) != ref).sum()),
          flush=True)
    assert ref.sum() > 300
    assert np.array_equal(dev, ref.astype(np.uint8))
    sim.step(7)
    dev = sim.read_interior()
    assert np.array_equal(dev, _oracle_mask(sim, w.lattice, w.tri).astype(np.uint8))


def test_marks_wrap_and_tile_edges():
    """Cells straddling periodic sides and tile boundaries, on a box whose
    sides are not multiples of the tile."""
    rest64, tri = rbc_mesh()
    rng = np.random.default_rng(43)
    lat = Lattice(29, 27, 21, tau=0.9)
    cen = np.array([[0.3, 13.2, 10.1], [14.6, 26.7, 3.2], [28.9, 1.1, 20.4]])
    rots = np.stack([random_rotation(rng) for _ in range(3)])
    cells = place_cells(rest64, cen, rots, np.ones((3, 4)) * 1e-3)
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri,
                                   cells=cells), cells)
    sim.init_equilibrium()
    sim.set_interior_viscosity(3.0)
    dev = sim.read_interior()
    ref = interior.inside_sites(cells.offsets, tri, (29, 27, 21), lat.bc, origin=cells.origin)
    assert ref.sum() > 600
    assert np.array_equal(dev, ref.astype(np.uint8))


@pytest.mark.parametrize("walls", [-1, 2])
def test_coupled_parity_interior_viscosity(walls):
    w = tiny_periodic(seed=44, n=(24, 22, 20), n_cells=2, walls=walls, body=(1e-5, 0, 0))
    rng = np.random.default_rng(45)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    sim.set_interior_viscosity(5.0)
    n = 12
    sim.step(4)
    sim.step(n - 4)
    sim.sync()
    m = step.make_model(w.lattice, w.rest_pos.astype(np.float64), w.tri, cells.k.astype(np.float64),
                        cells.traction.astype(np.float64), interior_ratio=5.0)
    f0, X0 = oracle_state(g0, cells)
    f, X = step.run(m, f0, X0, n)
    f_plain, _ = step.run(oracle_model(w, cells), f0, X0, n)
    o, off, _ = sim.read_vertices()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    effect = relerr(lattice.shifted(f_plain), lattice.shifted(f))
    Xg = o[:, None, :] + off.astype(np.float64)
    bound = n * 6e-8 * np.abs(off).max() + TOL * np.abs(X - X0).max()
    e_x = np.abs(Xg - X).max()
    print("walls", walls, "pops", e_g, "effect of the ratio", effect, "position", e_x, "bound", bound,
          flush=True)
    assert effect > 100 * TOL   # the interior relaxation changes the flow
    assert e_g <= TOL and e_x <= bound


def _class_bits(off, origin, tri, lat, ratios):
    """Expected mask bytes: 1 << k for the cells of the k-th smallest ratio,
    the highest k where cells overlap (the largest ratio wins, as in the
    oracle's ratio field)."""
    cls = np.searchsorted(np.unique(ratios), ratios)
    out = np.zeros((lat.nz, lat.ny, lat.nx), dtype=np.uint8)
    for c in range(len(ratios)):
        m = interior.inside_sites(off[c:c + 1], tri, (lat.nx, lat.ny, lat.nz), lat.bc,
                                  origin=origin[c:c + 1])
        out[m] = np.maximum(out[m], np.uint8(1 << cls[c]))
    return out


def test_per_cell_classes_marks_and_overlap():
    """Three viscosity classes; two cells of different classes overlap, and
    their shared sites carry the higher class, whatever the cell order."""
    rest64, tri = rbc_mesh()
    rng = np.random.default_rng(48)
    lat = Lattice(40, 32, 24, tau=0.9)
    cen = np.array([[10.2, 10.7, 11.4], [14.9, 11.3, 11.8], [29.6, 21.2, 12.3], [30.3, 5.1, 11.2]])
    rots = np.stack([random_rotation(rng) for _ in range(4)])
    cells = place_cells(rest64, cen, rots, np.ones((4, 4)) * 1e-3)
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri,
                                   cells=cells), cells)
    sim.init_equilibrium()
    ratios = np.array([5.0, 2.0, 5.0, 0.5], dtype=np.float32)
    sim.set_cell_viscosity(ratios)
    dev = sim.read_interior()
    ref = _class_bits(cells.offsets, cells.origin, tri, lat, ratios)
    print("bits", np.unique(ref, return_counts=True), flush=True)
    mA = interior.inside_sites(cells.offsets[:1], tri, (40, 32, 24), lat.bc, origin=cells.origin[:1])
    mB = interior.inside_sites(cells.offsets[1:2], tri, (40, 32, 24), lat.bc, origin=cells.origin[1:2])
    assert (mA & mB).sum() > 20           # overlap of a ratio-5 and a ratio-2 cell
    assert (ref[mA & mB] == 4).all()      # the ratio-5 class (k = 2) wins
    assert np.array_equal(dev, ref)
    # a new cell set returns to the single ratio (here never set: off)
    sim.set_cells(cells.origin, cells.offsets, cells.k, None)
    assert np.array_equal(sim.read_interior(), (ref > 0).astype(np.uint8))


def test_coupled_parity_per_cell_ratios():
    w = tiny_periodic(seed=49, n=(32, 24, 20), n_cells=3, walls=2, body=(1e-5, 0, 0))
    rng = np.random.default_rng(50)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    ratios = np.array([5.0, 10.0, 1.0])
    sim.set_cell_viscosity(ratios)
    n = 10
    sim.step(n)
    sim.sync()
    m = step.make_model(w.lattice, w.rest_pos.astype(np.float64), w.tri, cells.k.astype(np.float64),
                        cells.traction.astype(np.float64), interior_ratio=ratios)
    f0, X0 = oracle_state(g0, cells)
    f, X = step.run(m, f0, X0, n)
    o, off, _ = sim.read_vertices()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    Xg = o[:, None, :] + off.astype(np.float64)
    bound = n * 6e-8 * np.abs(off).max() + TOL * np.abs(X - X0).max()
    e_x = np.abs(Xg - X).max()
    print("pops", e_g, "position", e_x, "bound", bound, flush=True)
    assert e_g <= TOL and e_x <= bound


def test_ratio_one_and_refusals():
    w = tiny_periodic(seed=46, n=(24, 20, 16), n_cells=1)
    a, b = make_sim(w), make_sim(w)
    for s in (a, b):
        s.init_equilibrium()
    b.set_interior_viscosity(1.0)   # 1 switches the marking off: the same step bit for bit
    a.step(3)
    b.step(3)
    assert np.array_equal(a.read_populations(), b.read_populations())
    from paper_2305_02752_amd.hemo import HemoError
    with pytest.raises(HemoError, match="HC_ERR_ARG"):
        a.set_interior_viscosity(0.0)
    with pytest.raises(HemoError, match="HC_ERR_ARG"):
        a.set_interior_viscosity(float("nan"))
    a.set_cell_viscosity([1.0])   # one ratio for the one cell: accepted (and off)
    with pytest.raises(HemoError, match="HC_ERR_ARG"):
        a.set_cell_viscosity([2.0, 3.0])   # two ratios for one cell


def test_too_many_classes_refused():
    w = tiny_periodic(seed=51, n=(48, 48, 48), n_cells=9)
    sim = make_sim(w)
    from paper_2305_02752_amd.hemo import HemoError
    with pytest.raises(HemoError, match="HC_ERR_UNSUPPORTED"):
        sim.set_cell_viscosity(np.arange(9) + 1.0)
    sim.set_cell_viscosity(np.r_[np.arange(8) + 1.0, 2.0])   # 8 distinct: accepted


def test_no_cells_with_interior_viscosity():
    w = tiny_periodic(seed=47, n=(16, 16, 16), n_cells=1)
    from paper_2305_02752_amd import Simulation
    sim = Simulation(w.lattice, w.rest_pos, w.tri, max_cells=1)
    sim.init_equilibrium()
    sim.set_interior_viscosity(5.0)
    sim.step(2)
    assert not sim.read_interior().any()


def test_interior_with_separated_time_scales():
    """Interior viscosity combined with forces every 3 steps and
    Adams-Bashforth moves: the marks follow the moving cells every step."""
    from oracle import integrate
    w = tiny_periodic(seed=52, n=(24, 22, 20), n_cells=2, walls=1, body=(1e-5, 0, 0))
    rng = np.random.default_rng(53)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    sim.set_interior_viscosity(4.0)
    sim.set_integration(3, "ab2")
    n = 10
    sim.step(n)
    sim.sync()
    m = step.make_model(w.lattice, w.rest_pos.astype(np.float64), w.tri, cells.k.astype(np.float64),
                        cells.traction.astype(np.float64), interior_ratio=4.0)
    f0, X0 = oracle_state(g0, cells)
    f, X, _ = integrate.run(m, f0, X0, n, force_every=3, scheme="ab2")
    o, off, _ = sim.read_vertices()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    Xg = o[:, None, :] + off.astype(np.float64)
    bound = n * 6e-8 * np.abs(off).max() + TOL * np.abs(X - X0).max()
    e_x = np.abs(Xg - X).max()
    print("pops", e_g, "position", e_x, "bound", bound, flush=True)
    assert e_g <= TOL and e_x <= bound


def test_marks_of_a_stretched_cell_in_row_chunks():
    """A cell stretched along y to a bounding box of more than 320 columns
    is marked in several row chunks; the marks still match the oracle."""
    rest64, tri = rbc_mesh()
    lat = Lattice(40, 64, 24, tau=0.9)
    stretch = np.diag([1.0, 2.6, 1.0])
    from workloads.configs import place_cells as pc
    cells = pc(rest64 @ stretch.T, np.array([[19.3, 31.7, 11.4]]), np.eye(3)[None], np.ones((1, 4)) * 1e-3)
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri,
                                   cells=cells), cells)
    sim.init_equilibrium()
    sim.set_interior_viscosity(2.0)
    o, off = cells.origin, cells.offsets
    span = np.floor(off[0].max(0)) - np.ceil(off[0].min(0)) + 1
    assert span[0] * span[1] > 320          # more than one chunk
    dev = sim.read_interior()
    ref = interior.inside_sites(off, tri, (40, 64, 24), lat.bc, origin=o)
    assert ref.sum() > 1000
    assert np.array_equal(dev, ref.astype(np.uint8))


def _straddling_suspension(lat, seed, n=4):
    rest64, tri = rbc_mesh()
    rng = np.random.default_rng(seed)
    cen = np.column_stack([rng.uniform(0, lat.nx, n), rng.uniform(0, lat.ny, n),
                           np.where(np.arange(n) % 2 == 0, lat.nz - 0.7, 0.9) + rng.uniform(-0.4, 0.4, n)])
    rots = np.stack([random_rotation(rng) for _ in range(n)])
    k = np.ones((n, 4)) * 1e-3
    cells = jitter_cells(rng, place_cells(rest64, cen, rots, k, traction=np.zeros((n, 3))), 0.04)
    return rest64, tri, cells


def test_marks_with_sheared_images():
    """Lees-Edwards images: cells straddling z = 0 and z = nz are marked in
    the image above or below through their copies displaced by the image
    shift; bit-exact against the oracle's float32 local mode at the shift the
    device uses (fractional after a few steps)."""
    U = 0.037
    lat = Lattice(48, 32, 40, tau=1.0, lees_edwards_u=U)
    rest64, tri, cells = _straddling_suspension(lat, 54)
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri,
                                   cells=cells), cells)
    sim.init_equilibrium()
    sim.set_interior_viscosity(5.0)
    dims = (lat.nx, lat.ny, lat.nz)
    for steps in (0, 7):
        sim.step(steps)
        dev = sim.read_interior()
        o, off, _ = sim.read_vertices()
        n = sim.steps_taken()
        # the shift the device uses: U (float32) * n mod nx, in double, then float32
        d = np.float32(np.fmod(np.fmod(float(np.float32(U)) * n, lat.nx) + lat.nx, lat.nx))
        ref = interior.inside_sites(off, tri, dims, lat.bc, origin=o, le_delta=d)
        periodic = interior.inside_sites(off, tri, dims, lat.bc, origin=o)
        print("steps", n, "shift", d, "inside", int(ref.sum()), "differs from periodic",
              int((ref != periodic).sum()), flush=True)
        assert ref.sum() > 1000
        if n > 0:
            assert (ref != periodic).sum() > 50       # the images matter
        assert np.array_equal(dev, ref.astype(np.uint8))


def test_coupled_parity_sheared_images_with_interior_viscosity():
    U = 0.03
    lat = Lattice(40, 24, 32, tau=1.0, lees_edwards_u=U)
    rest64, tri, cells = _straddling_suspension(lat, 55, n=3)
    g0 = random_shifted_populations(np.random.default_rng(56), lat, 1e-3)
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri,
                                   cells=cells), cells)
    sim.write_populations(g0)
    sim.set_interior_viscosity(4.0)
    n = 6
    sim.step(n)
    sim.sync()
    m = step.make_model(lat, rest64, tri, cells.k.astype(np.float64), cells.traction.astype(np.float64),
                        le_u=U, interior_ratio=4.0)
    f0, X0 = oracle_state(g0, cells)
    f, X = step.run(m, f0, X0, n)
    plain, _ = step.run(step.make_model(lat, rest64, tri, cells.k.astype(np.float64),
                                        cells.traction.astype(np.float64), le_u=U), f0, X0, n)
    o, off, _ = sim.read_vertices()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    effect = relerr(lattice.shifted(plain), lattice.shifted(f))
    Xg = o[:, None, :] + off.astype(np.float64)
    bound = n * 6e-8 * np.abs(off).max() + TOL * np.abs(X - X0).max()
    e_x = np.abs(Xg - X).max()
    print("pops", e_g, "effect", effect, "position", e_x, "bound", bound, flush=True)
    assert effect > 100 * TOL
    assert e_g <= TOL and e_x <= bound
