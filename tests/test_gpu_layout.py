"""Device storage of the lattice: tile-major site order, pull-form state.

The library stores post-collision populations in 8^3-tile-major order and
converts at the C ABI.  These tests check the conversion on its own (a
write followed by a read is the identity, for periodic and walled lattices
with ragged tiles) and that switching the field output off changes nothing
but the read-out of the fields.
"""
import numpy as np
import pytest

from workloads import jitter_cells, random_shifted_populations, rbc_mesh, tiny_periodic
from workloads.configs import Lattice

from gpu_common import make_sim

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,walls", [((20, 12, 9), -1), ((13, 17, 10), 0), ((9, 8, 25), 1),
                                     ((16, 16, 16), 2), ((5, 6, 7), -1)])
def test_population_round_trip(n, walls):
    from paper_2305_02752_amd import Simulation
    bc = [0, 0, 0]
    if walls >= 0:
        bc[walls] = 1
    lat = Lattice(*n, bc=tuple(bc))
    rest, tri = rbc_mesh()
    g = random_shifted_populations(np.random.default_rng(22), lat, 1e-2)
    sim = Simulation(lat, rest.astype(np.float32), tri, max_cells=0)
    sim.write_populations(g)
    assert np.array_equal(sim.read_populations(), g)


def test_field_output_off_is_bitwise_identical():
    w = tiny_periodic(seed=23, n=(24, 20, 17), n_cells=2, walls=2)
    cells = jitter_cells(np.random.default_rng(24), w.cells, 0.05)
    g0 = random_shifted_populations(np.random.default_rng(25), w.lattice, 1e-3)
    outs = []
    for fields in (True, False):
        sim = make_sim(w, cells)
        sim.write_populations(g0)
        sim.set_field_output(fields)
        sim.step(5)
        sim.sync()
        outs.append((sim.read_populations(), sim.read_vertices()[1], sim.read_vertex_velocity()))
        if not fields:
            with pytest.raises(RuntimeError):
                sim.read_macro()
            with pytest.raises(RuntimeError):
                sim.read_force_field()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
