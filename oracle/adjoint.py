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
oracle run, dL/dp_j = (L(p + h e_j) - L(p - h e_j)) / 2h, h = eps |p_j|,
and independently by the complex-step method (cs_gradient).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import lattice, step


def extremes(X):
    """Indices of the vertices with the largest and smallest x and y (first
    index on ties; decided on the real part)."""
    R = np.real(X)
    return np.argmax(R[:, 0]), np.argmin(R[:, 0]), np.argmax(R[:, 1]), np.argmin(R[:, 1])


def diameters(X):
    """(D_A, D_T) of one cell's vertices X [V, 3]."""
    a, b, c, d = extremes(X)
    return X[a, 0] - X[b, 0], X[c, 1] - X[d, 1]


def loss_of(X, targets):
    da, dt = diameters(X)
    return (da - targets[0]) ** 2 + (dt - targets[1]) ** 2


def run_loss(lat, rest_pos, tri, X0, k, traction, tau, n, targets, f0=None, interior_ratio=1.0):
    """Loss after n oracle steps for one cell with stiffness k [4] and
    relaxation time tau (interior sites: tau_in = 1/2 + ratio (tau - 1/2))."""
    lat2 = dataclasses.replace(lat, tau=tau if np.iscomplexobj(tau) else float(tau))
    k = np.asarray(k)
    m = step.make_model(lat2, np.asarray(rest_pos, dtype=np.float64), tri,
                        k.astype(np.complex128 if np.iscomplexobj(k) else np.float64)[None],
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


def cs_gradient(lat, rest_pos, tri, X0, k, traction, tau, n, targets, f0=None, interior_ratio=1.0):
    """The same gradient by the complex-step method (Squire & Trapp 1998;
    Martins, Sturdza & Alonso 2003): dL/dp_j = Im L(p + i h e_j) / h with
    h = 1e-30 |p_j|.  The run is the oracle itself on complex numbers
    (forward-mode differentiation, one direction per run): no difference is
    taken, so the result is exact to float64 rounding, with no truncation
    error, independently of the finite differences.  Decisions (floor of a
    position, clamps, the extreme vertices) are taken on the real part."""
    p = np.concatenate([np.asarray(k, dtype=np.float64), [float(tau)]])
    g = np.zeros(5)
    for j in range(5):
        h = 1e-30 * abs(p[j])
        q = p.astype(np.complex128)
        q[j] += 1j * h
        L, _ = run_loss(lat, rest_pos, tri, X0, q[:4], traction, q[4], n, targets, f0=f0,
                        interior_ratio=interior_ratio)
        g[j] = L.imag / h
    return g
