"""Force-bias dense packing of surrogate ellipsoids (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.4: every cell is enclosed by an ellipsoid; the ellipsoids start at
random positions and orientations, and each iteration computes the overlap
of every pair and pushes overlapping pairs apart along the line through
their centres, with a magnitude proportional to the overlapping volume
(the pair force of Sec. 2.4: delta_ij p_ij times the unit vector between
the centres).  The scheme of the cited packing method is not in the paper.
Reading:

* ellipsoid i: centre r_i, rotation R_i (its columns are the body axes in
  the world frame) and semi-axes s_i; a point x lies inside when
  |diag(1 / s_i) R_i^T (x - r_i)| <= 1;
* the overlapping volume is estimated by quadrature: the points u_k are the
  centres of the m^3 cells of a regular grid over [-1, 1]^3 that lie in the
  unit ball (Q of them); ellipsoid i carries the points r_i + R_i (s_i u_k),
  each standing for V_i / Q of its volume.  With n_i(j) of i's points
  inside j, V_ij = (V_i n_i(j) + V_j n_j(i)) / (2 Q), symmetric in i and j;
* pairs whose bounding spheres (radius max s) do not meet are not tested;
* p_ij = V_ij and delta_ij = [V_ij > 0]; the displacement of i in one
  iteration is eta * sum_j V_ij (r_i - r_j) / |r_i - r_j| (a pair with
  coincident centres exerts none), shortened to max_move when longer; all
  ellipsoids move at once from the previous positions;
* periodic axes use the minimum image and wrap the centres into [0, L);
  on a wall axis the centre is clamped so that the ellipsoid's extent
  along the axis stays within [lo, hi];
* orientations stay fixed.

The inside tests can be taken in float32 (dtype) with each operation
rounded separately, which reproduces the integer decisions of a float32
implementation that evaluates the same expressions in the same order; all
other arithmetic is float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Domain:
    box: tuple            # sides L (x, y, z)
    periodic: tuple       # per axis: True periodic, False walls
    lo: tuple = (0.0, 0.0, 0.0)   # wall axes: allowed extent [lo, hi]
    hi: tuple = (0.0, 0.0, 0.0)


def unit_ball_points(m: int, dtype=np.float64) -> np.ndarray:
    """Centres of the m^3 grid cells over [-1, 1]^3 inside the unit ball, [Q, 3]."""
    g = (np.arange(m, dtype=dtype) * dtype(2) + dtype(1)) / dtype(m) - dtype(1)
    u = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    r2 = u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1] + u[:, 2] * u[:, 2]
    return u[r2 <= dtype(1)]


def min_image(d: np.ndarray, dom: Domain, dtype=np.float64) -> np.ndarray:
    """Separation vector(s) [..., 3] under the minimum-image convention."""
    out = np.array(d, dtype=dtype, copy=True)
    for a in range(3):
        if dom.periodic[a]:
            L = dtype(dom.box[a])
            out[..., a] = out[..., a] - L * np.rint(out[..., a] / L)
    return out


def count_inside(dd, Ri, si, Rj, sj, U):
    """n_i(j): how many of ellipsoid i's quadrature points lie in ellipsoid j.
    dd = r_i - r_j (minimum image); all arrays in one dtype, evaluated
    operation by operation.

    A point r_i + R_i (s_i u) lies in j when |t| <= 1 with
    t = diag(1/s_j) R_j^T (dd + R_i diag(s_i) u) = A u + b, where
    A = diag(1/s_j) (R_j^T R_i) diag(s_i) and b = diag(1/s_j) R_j^T dd are
    formed once per pair (left-to-right sums, reciprocals 1/s_j)."""
    one = dd.dtype.type(1)
    inv = [one / sj[e] for e in range(3)]
    M = [[(Rj[0, e] * Ri[0, c] + Rj[1, e] * Ri[1, c]) + Rj[2, e] * Ri[2, c] for c in range(3)]
         for e in range(3)]
    A = [[(M[e][c] * si[c]) * inv[e] for c in range(3)] for e in range(3)]
    b = [((Rj[0, e] * dd[0] + Rj[1, e] * dd[1]) + Rj[2, e] * dd[2]) * inv[e] for e in range(3)]
    t = [((A[e][0] * U[:, 0] + A[e][1] * U[:, 1]) + A[e][2] * U[:, 2]) + b[e] for e in range(3)]
    q = (t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]
    return int(np.count_nonzero(q <= one))


def volume(s) -> float:
    return 4.0 / 3.0 * np.pi * float(s[0]) * float(s[1]) * float(s[2])


def pair_overlaps(r, R, s, dom: Domain, m: int, dtype=np.float64):
    """Every pair i < j with bounding spheres that meet: list of
    (i, j, n_i(j), n_j(i), V_ij).  Brute force over all pairs."""
    r, R, s = np.asarray(r), np.asarray(R), np.asarray(s)
    U = unit_ball_points(m, dtype)
    Q = U.shape[0]
    rd, Rd, sd = r.astype(dtype), R.astype(dtype), s.astype(dtype)
    smax = sd.max(axis=1)
    out = []
    n = r.shape[0]
    for i in range(n):
        dd_all = min_image(rd[i][None, :] - rd, dom, dtype)
        d2 = dd_all[:, 0] * dd_all[:, 0] + dd_all[:, 1] * dd_all[:, 1] + dd_all[:, 2] * dd_all[:, 2]
        reach = smax[i] + smax
        for j in np.nonzero(d2 < reach * reach)[0]:
            if j <= i:
                continue
            nij = count_inside(dd_all[j], Rd[i], sd[i], Rd[j], sd[j], U)
            nji = count_inside(-dd_all[j], Rd[j], sd[j], Rd[i], sd[i], U)
            V = (volume(s[i]) * nij + volume(s[j]) * nji) / (2.0 * Q)
            out.append((i, int(j), nij, nji, V))
    return out


def extent(R, s) -> np.ndarray:
    """Half extent of each ellipsoid along each world axis, [n, 3]."""
    R = np.asarray(R, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    return np.sqrt(np.einsum("nde,ne->nd", R * R, s * s))


def iterate(r, R, s, dom: Domain, eta: float, max_move: float, m: int, dtype=np.float64):
    """One force-bias iteration: returns (new centres [n, 3] float64, pairs)."""
    r64 = np.asarray(r, dtype=np.float64)
    pairs = pair_overlaps(r, R, s, dom, m, dtype)
    disp = np.zeros_like(r64)
    for i, j, _, _, V in pairs:
        if V <= 0.0:
            continue
        d = min_image(r64[i] - r64[j], dom)
        nd = np.linalg.norm(d)
        if nd == 0.0:
            continue
        disp[i] += eta * V * d / nd
        disp[j] -= eta * V * d / nd
    ln = np.linalg.norm(disp, axis=1, keepdims=True)
    disp = np.where(ln > max_move, disp * (max_move / np.where(ln > 0, ln, 1.0)), disp)
    new = r64 + disp
    e = extent(R, s)
    for a in range(3):
        if dom.periodic[a]:
            new[:, a] = np.mod(new[:, a], dom.box[a])
        else:
            new[:, a] = np.minimum(np.maximum(new[:, a], dom.lo[a] + e[:, a]), dom.hi[a] - e[:, a])
    return new, pairs


def run(r, R, s, dom: Domain, eta: float, max_move: float, m: int, n_iter: int):
    """n_iter iterations from centres r (float64 arithmetic throughout)."""
    r = np.asarray(r, dtype=np.float64)
    for _ in range(n_iter):
        r, _ = iterate(r, R, s, dom, eta, max_move, m)
    return r


def residual(r, R, s, dom: Domain, m: int, dtype=np.float64):
    """(total overlapping volume sum_{i<j} V_ij, number of pairs with V_ij > 0)."""
    pairs = pair_overlaps(r, R, s, dom, m, dtype)
    return sum(p[4] for p in pairs), sum(1 for p in pairs if p[4] > 0.0)
