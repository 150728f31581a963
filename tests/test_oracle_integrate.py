"""Pins of the separated-time-scale cell integration (Sec. 2.6 reading).

* force_every = 1 with Euler is the plain coupled step, bit for bit;
* Euler and second-order Adams-Bashforth reproduce their closed-form
  trajectories in a uniformly accelerated periodic fluid: with a body force
  g on a fluid at rest the velocity carrying half the force is
  u^n = (n + 1/2) g exactly, so force-free vertices move by
  Euler: X^N - X^0 = g N^2 / 2,
  AB2:   X^N - X^0 = g (1/2 + N (N + 1) / 2 - 1)   (Euler first step);
* forces evaluated only at the rest shape and then held leave the cells
  passive tracers of the flow, unlike forces evaluated every step.
"""
import dataclasses

import numpy as np
import pytest

from oracle import integrate, lattice, step
from workloads import rbc_mesh
from workloads.configs import K_REF, Lattice, place_cells, small_rotation


def _model(lat, cells):
    rest64, tri = rbc_mesh()
    return step.make_model(lat, rest64, tri, cells.k.astype(np.float64),
                           None if cells.traction is None else cells.traction.astype(np.float64))


def _cell(lat, k, traction=None, seed=0):
    rest64, _ = rbc_mesh()
    rng = np.random.default_rng(seed)
    centre = np.array([(lat.nx - 1) / 2, (lat.ny - 1) / 2, (lat.nz - 1) / 2]) + rng.uniform(-0.4, 0.4, 3)
    return place_cells(rest64, centre[None], small_rotation(rng, 8.0)[None], np.asarray(k)[None],
                       traction=traction)


def test_force_every_one_euler_is_the_plain_step():
    lat = Lattice(20, 18, 16, bc=(0, 0, 1), tau=0.9, wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    cells = _cell(lat, K_REF, traction=[[2e-3, 0, 0]])
    m = _model(lat, cells)
    f0 = lattice.init_equilibrium(lat.shape)
    X0 = cells.positions64()
    f1, X1 = step.run(m, f0, X0, 4)
    f2, X2, st = integrate.run(m, f0, X0, 4, force_every=1, scheme="euler")
    assert np.array_equal(f1, f2) and np.array_equal(X1, X2) and st.steps == 4


@pytest.mark.parametrize("scheme", ["euler", "ab2"])
def test_closed_form_in_uniform_acceleration(scheme):
    g = 2e-5
    lat = Lattice(20, 20, 20, tau=0.8, body_force=(g, 0.0, 0.0))
    cells = _cell(lat, np.zeros(4))              # force-free cell
    m = _model(lat, cells)
    X0 = cells.positions64()
    N = 7
    _, XN, _ = integrate.run(m, lattice.init_equilibrium(lat.shape), X0, N, scheme=scheme)
    shift = g * N * N / 2 if scheme == "euler" else g * (0.5 + N * (N + 1) / 2 - 1)
    assert np.allclose(XN[..., 0] - X0[..., 0], shift, rtol=1e-9, atol=0)
    assert np.abs(XN[..., 1:] - X0[..., 1:]).max() < 1e-15


def test_forces_held_from_rest_shape_make_passive_tracers():
    lat = Lattice(24, 20, 20, bc=(0, 0, 1), tau=1.0, wall_u_lo=(-0.04, 0, 0), wall_u_hi=(0.04, 0, 0))
    rest64, tri = rbc_mesh()
    m = step.make_model(lat, rest64, tri, (K_REF * 10.0)[None])
    free = dataclasses.replace(m, k=np.zeros_like(m.k))
    f0 = lattice.init_equilibrium(lat.shape)
    X0 = rest64[None] + np.array([12.0, 10.0, 10.0])   # the rest shape itself, in float64
    n = 40
    _, X_held, _ = integrate.run(m, f0, X0, n, force_every=n, scheme="ab2")
    _, X_free, _ = integrate.run(free, f0, X0, n, force_every=1, scheme="ab2")
    _, X_live, _ = integrate.run(m, f0, X0, n, force_every=1, scheme="ab2")
    scale = np.abs(X_free - X0).max()
    assert np.abs(X_held - X_free).max() <= 1e-9 * scale
    assert np.abs(X_live - X_free).max() >= 1e-3 * scale
