"""Pins of the oracle's loss and finite-difference gradient.

The oracle gradient is central differences of the full FP64 run; these
tests show it is converged (step sizes a decade apart agree) and that the
loss seed (dL/dX at the extreme vertices) is the derivative of the loss.
"""
import numpy as np

from oracle import adjoint as oadj
from workloads import rbc_mesh
from workloads.configs import K_REF, Lattice, place_cells


def _setup():
    rest64, tri = rbc_mesh()
    lat = Lattice(20, 20, 20, bc=(0, 0, 1), tau=0.9, wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    cells = place_cells(rest64, np.array([[9.6, 9.3, 9.5]]), np.eye(3)[None], K_REF[None],
                        traction=[[3e-3, 0, 0]])
    return lat, rest64.astype(np.float32), tri, cells.positions64()[0], cells.traction[0]


def test_fd_gradient_converged():
    lat, rest, tri, X0, tr = _setup()
    targets = (19.0, 14.0)
    g3 = oadj.fd_gradient(lat, rest, tri, X0, K_REF, tr, lat.tau, 30, targets, eps=1e-3)
    g4 = oadj.fd_gradient(lat, rest, tri, X0, K_REF, tr, lat.tau, 30, targets, eps=1e-4)
    p = np.concatenate([K_REF, [lat.tau]])
    assert np.linalg.norm(p * g4) > 1e-3
    assert np.linalg.norm(p * (g3 - g4)) / np.linalg.norm(p * g4) < 1e-5


def test_loss_seed_is_loss_derivative():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(50, 3)) * 5
    t = (9.0, 7.0)
    da, dt = oadj.diameters(X)
    L = oadj.loss_of(X, t)
    assert abs(L - ((da - t[0]) ** 2 + (dt - t[1]) ** 2)) < 1e-12
    # derivative along x of the max-x vertex equals 2 (D_A - D_A*)
    i = int(np.argmax(X[:, 0]))
    h = 1e-6
    Xp = X.copy(); Xp[i, 0] += h
    Xm = X.copy(); Xm[i, 0] -= h
    assert abs((oadj.loss_of(Xp, t) - oadj.loss_of(Xm, t)) / (2 * h) - 2 * (da - t[0])) < 1e-6
