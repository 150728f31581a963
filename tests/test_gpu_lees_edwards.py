"""Lees-Edwards sheared periodic images on the device against the FP64 oracle
(Sec. 2.5 reading, oracle/lees_edwards.py).

* fluid only: populations after several steps with a growing image shift;
* coupled: one step (populations, force field, vertex velocity) and twelve
  steps (populations, positions) with a cell straddling the z boundary;
* a fluid-only box relaxes to the uniform shear the images impose;
* unsupported combinations are refused.
"""
import numpy as np
import pytest

from oracle import lattice, lees_edwards as le, step
from workloads import jitter_cells, random_shifted_populations, rbc_mesh
from workloads.configs import K_REF, Lattice, place_cells, small_rotation

from gpu_common import relerr

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5


def _sim(lat, cells=None, max_cells=None):
    from paper_2305_02752_amd import Simulation
    rest, tri = rbc_mesh()
    sim = Simulation(lat, rest.astype(np.float32), tri,
                     max_cells=max_cells if max_cells is not None else (cells.n if cells else 0))
    if cells is not None:
        sim.set_cells(cells.origin, cells.offsets, cells.k, cells.traction)
    return sim


def test_fluid_only_parity():
    U = 0.03
    lat = Lattice(16, 12, 24, tau=0.9, lees_edwards_u=U)
    g0 = random_shifted_populations(np.random.default_rng(41), lat, 1e-3)
    sim = _sim(lat)
    sim.write_populations(g0)
    n = 6
    sim.step(n)
    sim.sync()
    f = lattice.unshift(g0)
    F = np.zeros((3,) + lat.shape)
    for t in range(n):
        rho, u = lattice.moments(f, F)
        post = lattice.collide(f, rho, u, F, lat.tau)
        f = le.stream(post, U, le.image_shift(U, t, lat.nx))
    e = relerr(sim.read_populations(), lattice.shifted(f))
    print("fluid-only", e, flush=True)
    assert e <= n * TOL_STEP


def _straddling_cell(lat, seed):
    rest64, tri = rbc_mesh()
    rng = np.random.default_rng(seed)
    centre = np.array([lat.nx * 0.4, lat.ny * 0.5, lat.nz - 1.2]) + rng.uniform(-0.3, 0.3, 3)
    cells = place_cells(rest64, centre[None], small_rotation(rng, 10.0)[None],
                        (K_REF * 10.0 ** rng.uniform(-0.3, 0.3, 4))[None], traction=[[2e-3, 0, 0]])
    return rest64, tri, jitter_cells(rng, cells, 0.05)


def _oracle(lat, rest64, tri, cells, U):
    return step.make_model(lat, rest64, tri, cells.k.astype(np.float64), cells.traction.astype(np.float64),
                           le_u=U)


@pytest.mark.parametrize("U", [0.02, -0.035])
def test_coupled_one_step_parity(U):
    lat = Lattice(24, 20, 24, tau=1.0, lees_edwards_u=U)
    rest64, tri, cells = _straddling_cell(lat, 42)
    g0 = random_shifted_populations(np.random.default_rng(43), lat, 1e-3)
    sim = _sim(lat, cells)
    sim.write_populations(g0)
    sim.step(3)                      # the third step runs with image shift 2U
    sim.sync()
    m = _oracle(lat, rest64, tri, cells, U)
    f, X = lattice.unshift(g0), cells.positions64()
    for t in range(2):
        f, X, _ = step.step(m, f, X, t)
    f3, X3, info = step.step(m, f, X, 2)
    e_g = relerr(sim.read_populations(), lattice.shifted(f3))
    e_u = relerr(sim.read_vertex_velocity(), info["U"])
    print("coupled 3 steps", e_g, e_u, flush=True)
    assert e_g <= 3 * TOL_STEP and e_u <= 3 * TOL_STEP


def test_coupled_multistep_positions():
    U = 0.03
    lat = Lattice(24, 20, 24, tau=1.0, lees_edwards_u=U)
    rest64, tri, cells = _straddling_cell(lat, 44)
    sim = _sim(lat, cells)
    sim.init_equilibrium()
    n = 12
    sim.step(n)
    sim.sync()
    m = _oracle(lat, rest64, tri, cells, U)
    X0 = cells.positions64()
    f, X = step.run(m, lattice.init_equilibrium(lat.shape), X0, n)
    o, off, _ = sim.read_vertices()
    Xg = o[:, None, :] + off.astype(np.float64)
    bound = n * 6e-8 * np.abs(off).max() + 1e-4 * np.abs(X - X0).max()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    print("12 steps", e_g, np.abs(Xg - X).max(), bound, flush=True)
    assert e_g <= 1e-4 and np.abs(Xg - X).max() <= bound


def test_relaxes_to_uniform_shear():
    U = 0.02
    lat = Lattice(8, 8, 16, tau=1.0, lees_edwards_u=U)
    sim = _sim(lat)
    sim.init_equilibrium()
    sim.step(4000)
    sim.sync()
    rho, u = sim.read_macro()
    z = np.arange(lat.nz)
    exact = U * (z - (lat.nz - 1) / 2.0) / lat.nz
    prof = u[0].mean(axis=(1, 2))
    print("profile error", np.abs(prof - exact).max() / U, flush=True)
    assert np.abs(prof - exact).max() <= 1e-4 * U


def test_refused_combinations():
    from paper_2305_02752_amd import HemoError
    with pytest.raises(HemoError):
        _sim(Lattice(16, 16, 16, bc=(0, 1, 0), lees_edwards_u=0.01))
    with pytest.raises(HemoError):
        _sim(Lattice(20, 16, 16, lees_edwards_u=0.01))
    lat = Lattice(24, 20, 24, lees_edwards_u=0.01)
    _, _, cells = _straddling_cell(lat, 45)
    sim = _sim(lat, cells)
    with pytest.raises(HemoError):
        sim.adj_bind(10, 5)


def test_suspension_across_both_boundaries():
    """Eight cells, several straddling the sheared boundary at z = 0 and at
    z = nz and one crossing the x wrap as well, on a box of several tiles per
    axis: populations and positions after 6 steps, and the vertex velocity
    of the last step, against the FP64 oracle."""
    U = -0.025
    lat = Lattice(48, 32, 40, tau=0.95, lees_edwards_u=U)
    rest64, tri = rbc_mesh()
    rng = np.random.default_rng(45)
    cen = np.array([[10.3, 8.2, 0.6], [30.7, 20.4, 39.1], [47.6, 12.9, 1.4], [21.5, 27.3, 20.2],
                    [5.2, 25.1, 38.3], [38.9, 5.6, 12.7], [16.4, 15.8, 29.5], [42.1, 28.4, 0.2]])
    rots = np.stack([small_rotation(rng, 25.0) for _ in range(len(cen))])
    k = K_REF[None] * 10.0 ** rng.uniform(-0.3, 0.3, (len(cen), 4))
    cells = jitter_cells(rng, place_cells(rest64, cen, rots, k, traction=np.zeros((len(cen), 3))), 0.04)
    g0 = random_shifted_populations(rng, lat, 1e-3)
    sim = _sim(lat, cells)
    sim.write_populations(g0)
    n = 6
    sim.step(n)
    sim.sync()
    m = _oracle(lat, rest64, tri, cells, U)
    f, X = lattice.unshift(g0), cells.positions64()
    X0 = X.copy()
    for t in range(n):
        f, X, info = step.step(m, f, X, t)
    o, off, _ = sim.read_vertices()
    Xg = o[:, None, :] + off.astype(np.float64)
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    e_u = relerr(sim.read_vertex_velocity(), info["U"])
    bound = n * 6e-8 * np.abs(off).max() + 1e-4 * np.abs(X - X0).max()
    print("8 cells, 6 steps", e_g, e_u, np.abs(Xg - X).max(), bound, flush=True)
    assert e_g <= n * TOL_STEP and e_u <= n * TOL_STEP
    assert np.abs(Xg - X).max() <= bound


def test_sheared_touch_lists_bit_exact():
    # the device's tile lists with sheared images are the tiles holding at
    # least one of each vertex's stencil nodes, each node's x taken in its
    # own image (oracle binning), after several steps of a growing shift
    from oracle import binning
    U = 0.37   # a shift that is not a whole number of nodes
    lat = Lattice(32, 24, 32, tau=0.9, lees_edwards_u=U)
    _, _, cells = _straddling_cell(lat, 71)
    sim = _sim(lat, cells)
    sim.init_equilibrium()
    n = 9
    sim.step(n)
    sim.sync()
    sim.read_populations()   # brings the context's image shift to step n
    o, off, _ = sim.read_vertices()
    owner, tptr, touch, _, _ = sim.read_bins()
    t = n
    delta = np.float32(np.fmod(np.fmod(np.float64(np.float32(U)) * t, lat.nx) + lat.nx, lat.nx))
    ptr_r, vid_r = binning.touch_lists(o, off, (lat.nx, lat.ny, lat.nz), lat.bc, 4, le_delta=delta)
    # the cell straddles the boundary: some vertices reach two images
    assert np.any(np.floor(off[0, :, 2] + o[0, 2] - 1) < lat.nz) and np.any(off[0, :, 2] + o[0, 2] + 2 >= lat.nz)
    assert np.array_equal(tptr, ptr_r)
    assert np.array_equal(touch, vid_r)
