"""Cell-deformation loss and its FP64 gradient by central differences (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

The membrane parameters are fitted to single-cell stretching and shearing
measurements (Sec. 2.3), which makes the derivative of a cell-shape misfit
with respect to the stiffnesses and the relaxation time the quantity of
interest.  Reading of the loss: after n coupled steps,
    L = (D_A - D_A*)^2 + (D_T - D_T*)^2,
with D_A = max_v x - min_v x (axial extent) and D_T = max_v y - min_v y
(transverse extent) of the cell.  Parameters p = (k_link, k_bend, k_area,
k_volume, tau).  The gradient is central differences of the full FP64
oracle run, dL/dp_j = (L(p + h e_j) - L(p - h e_j)) / 2h, h = eps |p_j|.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import lattice, step


def diameters(X):
    """(D_A, D_T) of one cell's vertices X [V, 3]."""
    return X[:, 0].max() - X[:, 0].min(), X[:, 1].max() - X[:, 1].min()


def loss_of(X, targets):
    da, dt = diameters(X)
    return (da - targets[0]) ** 2 + (dt - targets[1]) ** 2


def run_loss(lat, rest_pos, tri, X0, k, traction, tau, n, targets, f0=None, interior_ratio=1.0):
    """Loss after n oracle steps for one cell with stiffness k [4] and
    relaxation time tau (interior sites: tau_in = 1/2 + ratio (tau - 1/2))."""
    lat2 = dataclasses.replace(lat, tau=float(tau))
    m = step.make_model(lat2, np.asarray(rest_pos, dtype=np.float64), tri,
                        np.asarray(k, dtype=np.float64)[None],
                        None if traction is None else np.asarray(traction, dtype=np.float64)[None],
                        interior_ratio=interior_ratio)
    f = lattice.init_equilibrium(lat.shape) if f0 is None else f0
    f, X = step.run(m, f, np.asarray(X0, dtype=np.float64)[None], n)
    return loss_of(X[0], targets), X[0]


def fd_gradient(lat, rest_pos, tri, X0, k, traction, tau, n, targets, eps=1e-4, f0=None,
                interior_ratio=1.0):
    """Central-difference gradient dL/d(k_link, k_bend, k_area, k_volume, tau)."""
    p = np.concatenate([np.asarray(k, dtype=np.float64), [float(tau)]])
    g = np.zeros(5)
    for j in range(5):
        h = eps * abs(p[j])
        vals = []
        for sgn in (+1.0, -1.0):
            q = p.copy()
            q[j] += sgn * h
            vals.append(run_loss(lat, rest_pos, tri, X0, q[:4], traction, q[4], n, targets, f0=f0,
                                 interior_ratio=interior_ratio)[0])
        g[j] = (vals[0] - vals[1]) / (2 * h)
    return g
