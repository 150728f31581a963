"""D3Q19 lattice-Boltzmann BGK with Guo forcing, in float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.2 gives the LBGK update f_i(x+e_i, t+1) = f_i + (f_i^eq - f_i)/tau,
the moments rho = sum f_i and u = sum f_i e_i / rho, the equilibrium
w_i rho [1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u^2], c_s = 1/sqrt(3) and
nu = c_s^2 (tau - 1/2).  Readings where the paper is silent:
  * direction order and weights: textbook D3Q19 (rest 1/3, axis 1/18,
    diagonal 1/36), order listed in `E` below, opposite of i>0 is i+1 for
    odd i and i-1 for even i;
  * external force (Sec. 2.3 couples through "external force terms"): Guo,
    Zheng & Shi (2002): u carries half the force, and the source term
    (1 - 1/(2 tau)) w_i [3 (e_i - u) + 9 (e_i.u) e_i].F is added;
  * walls: half-way bounce-back, wall half a lattice spacing outside the
    first/last fluid node, moving walls by Ladd's term -6 w_i rho (e_i.u_w).
Array layout: populations [19, nz, ny, nx], vectors [3, nz, ny, nx].
"""
from __future__ import annotations

import numpy as np

E = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
], dtype=np.int64)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
OPP = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, 19)])
CS2 = 1.0 / 3.0

PERIODIC = 0
WALL = 1


def equilibrium(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Second-order equilibrium of Sec. 2.2: w_i rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u]."""
    eu = np.tensordot(E.astype(np.float64), u, axes=(1, 0))          # [19, ...]
    uu = (u * u).sum(axis=0)
    w = W.reshape((19,) + (1,) * rho.ndim)
    return w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu)


def moments(f: np.ndarray, force: np.ndarray | None = None):
    """Density and velocity (Sec. 2.2 moments); with a force field the
    velocity includes half the force (Guo reading)."""
    rho = f.sum(axis=0)
    mom = np.tensordot(E.T.astype(np.float64), f, axes=(1, 0))        # [3, ...]
    if force is not None:
        mom = mom + 0.5 * force
    return rho, mom / rho


def guo_source(u: np.ndarray, force: np.ndarray, tau: float) -> np.ndarray:
    """Guo forcing term (1 - 1/(2 tau)) w_i [3 (e_i - u) + 9 (e_i.u) e_i] . F."""
    Ef = E.astype(np.float64)
    eu = np.tensordot(Ef, u, axes=(1, 0))                               # [19, ...]
    eF = np.tensordot(Ef, force, axes=(1, 0))
    uF = (u * force).sum(axis=0)
    w = W.reshape((19,) + (1,) * uF.ndim)
    return (1.0 - 0.5 / tau) * w * (3.0 * (eF - uF) + 9.0 * eu * eF)


def collide(f, rho, u, force, tau: float):
    """BGK relaxation toward equilibrium (Sec. 2.2 update) plus the Guo source."""
    feq = equilibrium(rho, u)
    post = f - (f - feq) / tau
    if force is not None:
        post = post + guo_source(u, force, tau)
    return post


def stream(post: np.ndarray, rho: np.ndarray, bc, wall_u_lo, wall_u_hi) -> np.ndarray:
    """Push streaming f_i(x + e_i) <- post_i(x) (left side of the Sec. 2.2
    update).  Periodic axes wrap.  On a wall axis a population that would
    leave the fluid returns to its own node in the opposite direction,
    minus Ladd's moving-wall term 6 w_i rho (e_i . u_wall)."""
    walls = [d for d in range(3) if bc[d] == WALL]
    if len(walls) > 1:
        raise NotImplementedError("at most one wall axis")
    out = np.empty_like(post)
    for i in range(19):
        out[i] = post[i]
        for d in range(3):
            if E[i, d] != 0:
                out[i] = np.roll(out[i], int(E[i, d]), axis=2 - d)
    for d in walls:
        ax = 2 - d
        n = post.shape[1 + ax]
        for i in range(19):
            if E[i, d] == 0:
                continue
            j = OPP[i]
            # population i arriving at the boundary layer from outside: it is the
            # bounce-back of population j that left this node through the wall.
            if E[i, d] > 0:
                layer, uw = 0, np.asarray(wall_u_lo, dtype=np.float64)
            else:
                layer, uw = n - 1, np.asarray(wall_u_hi, dtype=np.float64)
            sl = [slice(None)] * 3
            sl[ax] = layer
            sl = tuple(sl)
            ej_uw = float(E[j] @ uw)
            out[i][sl] = post[j][sl] - 6.0 * W[j] * rho[sl] * ej_uw
    return out


def lbm_step(f, force, tau, bc=(0, 0, 0), wall_u_lo=(0, 0, 0), wall_u_hi=(0, 0, 0)):
    """One fluid-only step: moments, collide, stream.  Returns (f_new, rho, u)."""
    rho, u = moments(f, force)
    post = collide(f, rho, u, force, tau)
    return stream(post, rho, bc, wall_u_lo, wall_u_hi), rho, u


def viscosity(tau: float) -> float:
    """Kinematic viscosity nu = c_s^2 (tau - 1/2) (Sec. 2.2)."""
    return CS2 * (tau - 0.5)


def init_equilibrium(shape, rho0=1.0, u0=(0.0, 0.0, 0.0)):
    rho = np.full(shape, float(rho0))
    u = np.empty((3,) + tuple(shape))
    for d in range(3):
        u[d] = u0[d]
    return equilibrium(rho, u)


def shifted(f):
    """Shifted populations g_i = f_i - w_i (the stored form on the device)."""
    return f - W.reshape((19,) + (1,) * (f.ndim - 1))


def unshift(g):
    return np.asarray(g, dtype=np.float64) + W.reshape((19,) + (1,) * (g.ndim - 1))
