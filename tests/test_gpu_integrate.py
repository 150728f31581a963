"""Separated cell time scales on the device against the FP64 oracle.

Membrane forces every `force_every` steps (held in between) and Euler or
second-order Adams-Bashforth moves (Sec. 2.6 reading, oracle/integrate.py).
Bars: populations within 1e-4 after 12 steps (1e-5 per step accumulated),
positions within the same fraction of the displacement plus the rounding
of the float32 offsets (half an ulp per move); closed-form AB2 trajectory in a uniformly
accelerated fluid; bitwise resume from a checkpoint taken inside a
force-refresh interval.
"""
import numpy as np
import pytest

from oracle import integrate, lattice
from workloads import jitter_cells, random_shifted_populations, rbc_mesh, tiny_periodic
from workloads.configs import Lattice, place_cells, small_rotation

from gpu_common import make_sim, oracle_model, oracle_state, relerr

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.mark.parametrize("force_every,scheme,walls", [(1, "ab2", 2), (3, "euler", -1), (4, "ab2", 1),
                                                      (5, "ab2", -1)])
def test_separated_time_scales_parity(force_every, scheme, walls):
    w = tiny_periodic(seed=31, n=(24, 22, 20), n_cells=2, walls=walls, body=(1e-5, 0, 0))
    rng = np.random.default_rng(32)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    sim.set_integration(force_every, scheme)
    n = 12
    sim.step(5)
    sim.step(n - 5)       # two calls: the pending move crosses a call boundary
    sim.sync()
    m = oracle_model(w, cells)
    f0, X0 = oracle_state(g0, cells)
    f, X, _ = integrate.run(m, f0, X0, n, force_every=force_every, scheme=scheme)
    o, off, _ = sim.read_vertices()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    Xg = o[:, None, :] + off.astype(np.float64)
    # positions are float32 offsets: each move rounds by at most half an ulp
    bound = n * 6e-8 * np.abs(off).max() + TOL * np.abs(X - X0).max()
    e_x = np.abs(Xg - X).max()
    print(force_every, scheme, walls, "pops", e_g, "position error", e_x, "bound", bound, flush=True)
    assert e_g <= TOL and e_x <= bound


def test_ab2_closed_form_uniform_acceleration():
    g = 2e-5
    lat = Lattice(24, 24, 24, tau=0.8, body_force=(g, 0.0, 0.0))
    rest64, tri = rbc_mesh()
    rng = np.random.default_rng(33)
    cells = place_cells(rest64, np.array([[11.3, 11.7, 12.2]]), small_rotation(rng, 8.0)[None],
                        np.zeros((1, 4)))
    from paper_2305_02752_amd import Simulation
    sim = Simulation(lat, rest64.astype(np.float32), tri, max_cells=1)
    sim.set_cells(cells.origin, cells.offsets, cells.k, None)
    sim.init_equilibrium()
    sim.set_integration(1, "ab2")
    N = 9
    sim.step(N)
    sim.sync()
    o, off, _ = sim.read_vertices()
    X = o[:, None, :] + off.astype(np.float64)
    X0 = cells.positions64()
    shift = g * (0.5 + N * (N + 1) / 2 - 1)
    # each move rounds the float32 offset by at most half an ulp (<= 6e-8 |offset|)
    rounding = N * 6e-8 * np.abs(off).max()
    assert np.abs(X[..., 0] - X0[..., 0] - shift).max() <= 1e-5 * shift + rounding
    assert np.abs(X[..., 1:] - X0[..., 1:]).max() <= rounding


def test_resume_inside_refresh_interval_bitwise():
    w = tiny_periodic(seed=34, n=(24, 20, 20), n_cells=2, walls=2)
    cells = jitter_cells(np.random.default_rng(35), w.cells, 0.05)
    sim = make_sim(w, cells)
    sim.set_integration(4, "ab2")
    sim.step(6)                  # two steps into a refresh interval
    ck = sim.checkpoint_save()
    sim.step(7)
    sim.sync()
    ref = (sim.read_populations(), sim.read_vertices()[1], sim.read_vertex_velocity())
    sim2 = make_sim(w, cells)
    sim2.checkpoint_restore(ck)
    sim2.step(7)
    sim2.sync()
    for a, b in zip(ref, (sim2.read_populations(), sim2.read_vertices()[1], sim2.read_vertex_velocity())):
        assert np.array_equal(a, b)


def test_adjoint_refuses_separated_time_scales():
    from paper_2305_02752_amd import HemoError
    w = tiny_periodic(seed=36, n=(20, 20, 20), n_cells=1)
    sim = make_sim(w)
    sim.set_integration(2, "euler")
    with pytest.raises(HemoError):
        sim.adj_bind(10, 5)
