"""One coupled fluid-cell time step, float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.3 couples the fluid and the cells explicitly through external force
terms with interpolation in both directions; Sec. 2.6 integrates the cells
with explicit Euler.  The paper does not fix the order inside a step; the
reading used here is:
  1. membrane forces F_v from the positions X^n (Sec. 2.3 force sum);
  2. Eulerian force density F(x) = body force + spread of F_v (Sec. 2.3);
  3. moments rho^n, u^n of f^n with half the force (Sec. 2.2, Guo reading);
  4. vertex velocity U_v interpolated from u^n (Sec. 2.3);
  5. BGK collision with the Guo source, then streaming (Sec. 2.2 update);
  6. X^{n+1} = X^n + U_v (explicit Euler, Sec. 2.6).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import ibm, interior, lattice, lees_edwards, membrane


@dataclasses.dataclass
class Model:
    dims: tuple            # (nx, ny, nz)
    bc: tuple
    tau: float
    body_force: tuple
    wall_u_lo: tuple
    wall_u_hi: tuple
    kernel: int
    topo: membrane.Topology
    rest: membrane.RestState
    k: np.ndarray          # [C, 4]
    traction: np.ndarray | None
    le_u: float = 0.0      # Lees-Edwards image velocity along x (gradient axis z); 0: off
    interior_ratio: float | np.ndarray = 1.0   # viscosity ratio inside the cells, one or per cell (1: off)


def make_model(lat, rest_pos, tri, k, traction=None, le_u: float = 0.0,
               interior_ratio=1.0) -> Model:
    topo = membrane.Topology(tri, rest_pos.shape[0])
    rest = membrane.RestState(np.asarray(rest_pos, dtype=np.float64), topo)
    # tau and k stay complex when the complex-step gradient perturbs them
    tau = complex(lat.tau) if np.iscomplexobj(lat.tau) else float(lat.tau)
    k = np.asarray(k)
    k = k.astype(np.complex128 if np.iscomplexobj(k) else np.float64)
    return Model(dims=(lat.nx, lat.ny, lat.nz), bc=tuple(lat.bc), tau=tau,
                 body_force=tuple(float(b) for b in lat.body_force),
                 wall_u_lo=tuple(lat.wall_u_lo), wall_u_hi=tuple(lat.wall_u_hi),
                 kernel=int(lat.ibm_kernel), topo=topo, rest=rest,
                 k=k,
                 traction=None if traction is None else np.asarray(traction, dtype=np.float64),
                 le_u=float(le_u),
                 interior_ratio=(float(interior_ratio) if np.ndim(interior_ratio) == 0
                                 else np.asarray(interior_ratio, dtype=np.float64)))


def fluid_step(m: Model, f: np.ndarray, X: np.ndarray, Fv: np.ndarray, t: int = 0):
    """Steps 2-5 with given vertex forces Fv [C, V, 3]: returns the streamed
    populations, the interpolated vertex velocity U and the intermediate
    fields.  t: the step index (fixes the Lees-Edwards image shift)."""
    nx, ny, nz = m.dims
    C = X.shape[0]
    le = m.le_u != 0.0
    delta = lees_edwards.image_shift(m.le_u, t, nx) if le else 0.0
    if C and le:
        F = lees_edwards.spread(X.reshape(-1, 3), Fv.reshape(-1, 3), m.dims, delta, m.kernel)
    elif C:
        F = ibm.spread(X.reshape(-1, 3), Fv.reshape(-1, 3), m.dims, m.bc, m.kernel)
    else:
        F = np.zeros((3, nz, ny, nx), dtype=f.dtype)
    for d in range(3):
        F[d] += m.body_force[d]
    rho, u = lattice.moments(f, F)
    if C and le:
        U = lees_edwards.interpolate(u, X.reshape(-1, 3), m.dims, m.le_u, delta,
                                     m.kernel).reshape(X.shape)
    elif C:
        U = ibm.interpolate(u, X.reshape(-1, 3), m.dims, m.bc, m.wall_u_lo, m.wall_u_hi,
                            m.kernel).reshape(X.shape)
    else:
        U = np.zeros_like(X)
    tau = m.tau
    ratios = np.broadcast_to(np.asarray(m.interior_ratio, dtype=np.float64), (C,))
    if C and np.any(ratios != 1.0):   # inside/outside is decided on the real positions
        tau = interior.tau_field(interior.ratio_field(np.real(X), m.topo.tri, m.dims, m.bc, ratios,
                                                      le_delta=delta if le else 0.0), m.tau)
    post = lattice.collide(f, rho, u, F, tau)
    if le:
        f_new = lees_edwards.stream(post, m.le_u, delta)
    else:
        f_new = lattice.stream(post, rho, m.bc, m.wall_u_lo, m.wall_u_hi)
    return f_new, U, {"Fv": Fv, "F": F, "rho": rho, "u": u, "U": U}


def step(m: Model, f: np.ndarray, X: np.ndarray, t: int = 0):
    """Advance populations f [19, nz, ny, nx] and positions X [C, V, 3] by one
    step (t: its index, counted from 0).

    Returns (f_new, X_new, info) where info holds the intermediate fields.
    """
    Fv = membrane.forces(X, m.k, m.topo, m.rest, m.traction) if X.shape[0] else np.zeros_like(X)
    f_new, U, info = fluid_step(m, f, X, Fv, t)
    return f_new, X + U, info


def run(m: Model, f, X, n: int, t0: int = 0):
    for i in range(n):
        f, X, _ = step(m, f, X, t0 + i)
    return f, X
