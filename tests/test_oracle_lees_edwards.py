"""Pins of the Lees-Edwards oracle (Sec. 2.5 reading, oracle/lees_edwards.py).

* U = 0 and Delta = 0: the periodic streaming (to rounding);
* U = 0 and an integer Delta: the populations crossing the z boundary are
  the neighbouring rows shifted by Delta columns, nothing else changes;
* mass is conserved exactly for any Delta and U (linear interpolation along
  a periodic row and the Galilean term both keep it);
* a fluid-only box relaxes to the uniform shear u_x = U (z - (nz - 1)/2) / nz
  that the sheared images impose (the discrete solution of Couette flow is
  linear);
* a vertex straddling the boundary interpolates an image-consistent linear
  shear field exactly, and spreading keeps its total force.
"""
import numpy as np
import pytest

from oracle import lattice, lees_edwards as le


def _random_post(rng, shape):
    f = lattice.init_equilibrium(shape)
    return f + 1e-3 * rng.standard_normal(f.shape)


def test_zero_shear_is_periodic_streaming():
    rng = np.random.default_rng(1)
    post = _random_post(rng, (12, 6, 10))
    rho = post.sum(axis=0)
    ref = lattice.stream(post, rho, (0, 0, 0), (0, 0, 0), (0, 0, 0))
    assert np.allclose(le.stream(post, 0.0, 0.0), ref, rtol=0, atol=1e-15)


def test_integer_shift_moves_boundary_rows():
    rng = np.random.default_rng(2)
    nz, ny, nx = 10, 6, 12
    post = _random_post(rng, (nz, ny, nx))
    k = 5
    out = le.stream(post, 0.0, float(k))
    rho = post.sum(axis=0)
    per = lattice.stream(post, rho, (0, 0, 0), (0, 0, 0), (0, 0, 0))
    for i in range(19):
        ez = lattice.E[i, 2]
        ref = per[i].copy()
        if ez > 0:     # row 0 receives the top row of the image below, displaced by -k
            ref[0] = np.roll(per[i][0], -k, axis=1)
        if ez < 0:
            ref[nz - 1] = np.roll(per[i][nz - 1], k, axis=1)
        assert np.allclose(out[i], ref, rtol=0, atol=1e-15), i


@pytest.mark.parametrize("delta,u", [(3.37, 0.02), (11.9, -0.05), (0.5, 0.1)])
def test_mass_conserved(delta, u):
    rng = np.random.default_rng(3)
    post = _random_post(rng, (8, 5, 12))
    out = le.stream(post, u, delta)
    assert abs(out.sum() - post.sum()) <= 1e-12 * post.sum()


def test_relaxes_to_uniform_shear():
    nx, ny, nz = 4, 4, 16
    U, tau = 0.02, 1.0
    f = lattice.init_equilibrium((nz, ny, nx))
    F = np.zeros((3, nz, ny, nx))
    for t in range(4000):
        rho, u = lattice.moments(f, F)
        post = lattice.collide(f, rho, u, F, tau)
        f = le.stream(post, U, le.image_shift(U, t, nx))
    rho, u = lattice.moments(f, F)
    z = np.arange(nz)
    exact = U * (z - (nz - 1) / 2.0) / nz
    prof = u[0].mean(axis=(1, 2))
    assert np.abs(prof - exact).max() <= 1e-8 * U
    assert np.abs(u[0] - prof[:, None, None]).max() <= 1e-12
    assert np.abs(u[1:]).max() <= 1e-12
    assert abs(rho.mean() - 1.0) <= 1e-12


def test_ibm_across_the_boundary():
    nx, ny, nz = 16, 12, 16
    U, delta = 0.04, 5.3
    gamma = U / nz
    z = np.arange(nz, dtype=np.float64)
    u = np.zeros((3, nz, ny, nx))
    u[0] = gamma * (z - 3.0)[:, None, None]
    X = np.array([[4.3, 6.7, 15.6], [9.1, 2.2, 0.4], [15.7, 11.5, 16.2], [0.2, 5.5, -0.8]])
    Ui = le.interpolate(u, X, (nx, ny, nz), U, delta)
    assert np.allclose(Ui[:, 0], gamma * (X[:, 2] - 3.0), rtol=0, atol=1e-15)
    assert np.abs(Ui[:, 1:]).max() <= 1e-15
    Fv = np.array([[1.0, -2.0, 0.5], [0.3, 0.1, -0.7], [2.0, 1.0, 1.0], [-1.0, 0.0, 3.0]])
    Fl = le.spread(X, Fv, (nx, ny, nz), delta)
    assert np.allclose(Fl.reshape(3, -1).sum(axis=1), Fv.sum(axis=0), rtol=0, atol=1e-13)
