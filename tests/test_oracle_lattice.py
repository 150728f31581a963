"""Pins of the lattice oracle against closed forms and exact invariants.

Sec. 2.2 fixes the LBGK update, the moments, the equilibrium, c_s^2 = 1/3
and nu = c_s^2 (tau - 1/2); the tests below check the oracle against
textbook consequences of those statements that do not reuse its code.
"""
import json
import os

import numpy as np
import pytest

from oracle import lattice as L

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_velocity_set_isotropy():
    """Lattice tensors of D3Q19: sum w = 1, sum w e = 0, sum w e e = cs2 I,
    sum w e e e e = cs2^2 (d d + d d + d d) -- fixes weights and directions."""
    E = L.E.astype(float)
    cs2 = GOLD["cs2"]["value"]
    assert abs(L.W.sum() - 1) < 1e-15
    assert np.abs(L.W @ E).max() < 1e-15
    T2 = np.einsum("i,ia,ib->ab", L.W, E, E)
    assert np.allclose(T2, cs2 * np.eye(3), atol=1e-15)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", L.W, E, E, E, E)
    d = np.eye(3)
    iso = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(T4, iso, atol=1e-15)
    assert len({tuple(e) for e in L.E}) == 19
    assert all((L.E[L.OPP[i]] == -L.E[i]).all() for i in range(19))


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho = 1 + 0.05 * rng.standard_normal((4, 5, 6))
    u = 0.05 * rng.standard_normal((3, 4, 5, 6))
    feq = L.equilibrium(rho, u)
    E = L.E.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=0, atol=1e-14)
    assert np.allclose(np.tensordot(E.T, feq, 1), rho * u, atol=1e-14)
    P = np.einsum("ia,ib,i...->ab...", E, E, feq)
    ref = rho * (np.eye(3)[:, :, None, None, None] / 3.0 + u[:, None] * u[None, :])
    assert np.allclose(P, ref, atol=1e-14)


def test_guo_source_moments():
    """Guo source: zero mass, momentum (1 - 1/(2 tau)) F."""
    rng = np.random.default_rng(1)
    u = 0.03 * rng.standard_normal((3, 7))
    F = 1e-3 * rng.standard_normal((3, 7))
    for tau in (0.6, 1.0, 1.9):
        S = L.guo_source(u, F, tau)
        assert np.abs(S.sum(0)).max() < 1e-18
        assert np.allclose(np.tensordot(L.E.T.astype(float), S, 1), (1 - 0.5 / tau) * F, atol=1e-18)


def test_stream_moves_each_population_by_its_velocity():
    shape = (5, 6, 7)
    post = np.zeros((19,) + shape)
    post[:, 2, 3, 4] = np.arange(19) + 1.0
    out = L.stream(post, np.ones(shape), (0, 0, 0), (0, 0, 0), (0, 0, 0))
    for i in range(19):
        ex, ey, ez = L.E[i]
        z, y, x = (2 + ez) % 5, (3 + ey) % 6, (4 + ex) % 7
        assert out[i, z, y, x] == i + 1
        assert out[i].sum() == i + 1


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_couette_exact(tau):
    """Steady Couette flow between walls moving at -+u_w is exactly linear
    with half-way bounce-back: u_x(z) = u_w (2 (z + 1/2)/N - 1)."""
    nz = 24
    f = L.init_equilibrium((nz, 1, 1))
    for _ in range(12000):
        f, _, _ = L.lbm_step(f, None, tau, bc=(0, 0, 1), wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    _, u = L.moments(f)
    z = np.arange(nz)
    assert np.abs(u[0, :, 0, 0] - 0.01 * (2 * (z + 0.5) / nz - 1)).max() < 1e-12


def test_poiseuille_magic_tau_exact():
    """Body-force channel: u(y) = g/(2 nu) (y + 1/2)(N - 1/2 - y) with
    nu = cs2 (tau - 1/2); exact for BGK at Lambda = (tau - 1/2)^2 = 3/16."""
    ny, g = 16, 1e-5
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    f = L.init_equilibrium((1, ny, 1))
    F = np.zeros((3, 1, ny, 1))
    F[0] = g
    for _ in range(25000):
        f, _, _ = L.lbm_step(f, F, tau, bc=(0, 1, 0))
    _, u = L.moments(f, F)
    nu = eval(GOLD["viscosity"]["formula"], {"cs2": GOLD["cs2"]["value"], "tau": tau})
    y = np.arange(ny)
    ex = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    assert np.abs(u[0, 0, :, 0] - ex).max() / ex.max() < 1e-9


def test_poiseuille_bulk_curvature_tau1():
    """At tau = 1 the interior second difference equals -g/nu exactly."""
    ny, g, tau = 16, 1e-5, 1.0
    f = L.init_equilibrium((1, ny, 1))
    F = np.zeros((3, 1, ny, 1))
    F[0] = g
    for _ in range(20000):
        f, _, _ = L.lbm_step(f, F, tau, bc=(0, 1, 0))
    _, u = L.moments(f, F)
    ux = u[0, 0, :, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    assert np.allclose(d2, -g / L.viscosity(tau), rtol=1e-8)


def test_shear_wave_decay_gives_viscosity():
    """A shear wave u_x = A sin(k z) decays at the rate nu k^2 with
    nu = cs2 (tau - 1/2) (Sec. 2.2)."""
    nz, tau, A = 64, 0.8, 1e-4
    z = np.arange(nz)
    k = 2 * np.pi / nz
    u = np.zeros((3, nz, 1, 1))
    u[0, :, 0, 0] = A * np.sin(k * z)
    f = L.equilibrium(np.ones((nz, 1, 1)), u)
    n = 400
    for _ in range(n):
        f, _, _ = L.lbm_step(f, None, tau)
    _, u1 = L.moments(f)
    amp = 2 * np.mean(u1[0, :, 0, 0] * np.sin(k * z))
    nu_meas = -np.log(amp / A) / (k * k * n)
    assert abs(nu_meas / L.viscosity(tau) - 1) < 5e-3


def test_mass_exact_with_moving_walls():
    rng = np.random.default_rng(2)
    shape = (8, 6, 5)
    f = L.init_equilibrium(shape) + 1e-3 * rng.standard_normal((19,) + shape)
    m0 = f.sum()
    for _ in range(50):
        f, _, _ = L.lbm_step(f, None, 0.9, bc=(0, 0, 1), wall_u_lo=(-0.01, 0.005, 0), wall_u_hi=(0.01, 0, 0))
    assert abs(f.sum() - m0) < 1e-11


def test_momentum_identity_with_guo_forcing():
    """Periodic box: total momentum after a step = before + sum of F."""
    rng = np.random.default_rng(3)
    shape = (6, 5, 7)
    f = L.init_equilibrium(shape) + 1e-3 * rng.standard_normal((19,) + shape)
    F = 1e-4 * rng.standard_normal((3,) + shape)
    E = L.E.T.astype(float)
    p0 = np.tensordot(E, f, 1).sum(axis=(1, 2, 3))
    f1, _, _ = L.lbm_step(f, F, 0.75)
    p1 = np.tensordot(E, f1, 1).sum(axis=(1, 2, 3))
    assert np.allclose(p1 - p0, F.sum(axis=(1, 2, 3)), atol=1e-14)


def test_rest_state_is_fixed_point():
    f = L.init_equilibrium((4, 4, 4))
    f1, _, _ = L.lbm_step(f, None, 1.3, bc=(0, 1, 0))
    assert np.abs(f1 - f).max() < 1e-16
