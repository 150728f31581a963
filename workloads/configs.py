"""Seeded synthetic workloads standing in for the paper's cell-suspension runs.

The paper's applications (straight and curved vessels, stiffened-cell pipe
flow, single-cell shearing and stretching; Sec. 3 and Sec. 2.3) need
geometries and measured data that are not available, so each workload below
is a synthetic input with the lattice size, boundary conditions, cell count,
haematocrit and parameter spread of the run it stands in for.  All draws use
numpy's PCG64 generator (`numpy.random.default_rng(seed)`).

Units are lattice units (dx = 0.5 um).  Positions are handed over as a
per-cell integer origin plus float32 offsets; the oracle promotes the same
float32 values to float64.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .mesh import rbc_mesh

PERIODIC = 0
WALL = 1

# Reference membrane stiffnesses (link, bend, area, volume) in lattice units.
K_REF = np.array([1.5e-4, 1.0e-5, 5.0e-2, 1.0e-2], dtype=np.float64)
# 200 pN expressed in lattice force units (dx = 0.5 um, dt = 3.79e-8 s, rho = 1025 kg/m^3).
PN200_LU = 4.48e-3


@dataclasses.dataclass
class Lattice:
    nx: int
    ny: int
    nz: int
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    tau: float = 1.0
    body_force: tuple = (0.0, 0.0, 0.0)
    wall_u_lo: tuple = (0.0, 0.0, 0.0)
    wall_u_hi: tuple = (0.0, 0.0, 0.0)
    ibm_kernel: int = 4          # 4: Peskin 4-point, 2: linear hat
    lees_edwards_u: float = 0.0  # sheared periodic images along x across z (0: off)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_sites(self):
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Cells:
    origin: np.ndarray      # int32 [C,3]
    offsets: np.ndarray     # float32 [C,V,3]
    k: np.ndarray           # float32 [C,4]  link, bend, area, volume
    traction: np.ndarray | None = None   # float32 [C,3] pole traction vector

    @property
    def n(self):
        return int(self.origin.shape[0])

    def positions64(self):
        """Absolute positions as float64 (origin + promoted float32 offsets)."""
        return self.origin[:, None, :].astype(np.float64) + self.offsets.astype(np.float64)


@dataclasses.dataclass
class Workload:
    name: str
    lattice: Lattice | list
    rest_pos: np.ndarray     # float32 [V,3]
    tri: np.ndarray          # int32 [T,3]
    cells: Cells | list
    steps: int
    extra: dict = dataclasses.field(default_factory=dict)


# --------------------------------------------------------------------------- rotations
def random_rotation(rng) -> np.ndarray:
    """Uniform random rotation matrix from a uniform unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    q = np.array([a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2),
                  b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)])
    return _quat_to_matrix(q)


def small_rotation(rng, max_deg: float) -> np.ndarray:
    """Rotation by an angle U(0, max_deg) about a uniformly random axis."""
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    ang = math.radians(rng.uniform(0.0, max_deg))
    q = np.concatenate([ax * math.sin(ang / 2), [math.cos(ang / 2)]])
    return _quat_to_matrix(q)


def _quat_to_matrix(q):
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# --------------------------------------------------------------------------- placement
def place_cells(rest64: np.ndarray, centres: np.ndarray, rots: np.ndarray,
                k: np.ndarray, traction=None) -> Cells:
    """Rigidly place the rest mesh at each centre with each rotation.

    The integer origin is floor(centre); offsets are rounded to float32.
    """
    C = centres.shape[0]
    X = np.einsum("cij,vj->cvi", rots, rest64) + centres[:, None, :]
    origin = np.floor(centres).astype(np.int32)
    off = (X - origin[:, None, :]).astype(np.float32)
    tr = None if traction is None else np.asarray(traction, dtype=np.float32).reshape(C, 3)
    return Cells(origin=origin, offsets=off, k=np.asarray(k, dtype=np.float32).reshape(C, 4), traction=tr)


def log_uniform_k(rng, n: int) -> np.ndarray:
    """Per-cell stiffnesses, each log-uniform over one decade centred on K_REF."""
    e = rng.uniform(-0.5, 0.5, size=(n, 4))
    return K_REF[None, :] * 10.0 ** e


def _mesh():
    rest64, tri = rbc_mesh(3, 16.0)
    return rest64, tri


# --------------------------------------------------------------------------- packing
def _surrogate_spheres():
    """Sphere cluster covering the biconcave cell in its own frame.

    One sphere on the axis and twelve on a ring in the disk plane.  The
    force-bias packing below acts on these clusters instead of on exact
    ellipsoids (a cheaper surrogate of the same kind).
    """
    pts = [np.zeros(3)]
    for m in range(12):
        a = 2 * math.pi * m / 12
        pts.append(np.array([5.4 * math.cos(a), 5.4 * math.sin(a), 0.0]))
    return np.array(pts), 2.7


# Semi-axes of an oblate ellipsoid enclosing the rest mesh (radius 8, half
# thickness 2.62 at the rim of the dimple): every vertex satisfies
# (r / 8.5)^2 + (z / 3.8)^2 <= 1.
RBC_SURROGATE = (8.5, 8.5, 3.8)


def random_rotations(rng, n: int) -> np.ndarray:
    """n uniform random rotations [n, 3, 3] from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)


def ellipsoid_suspension(seed: int = 6, n: int = 1_000_000, fraction: float = 0.35,
                         semi=RBC_SURROGATE):
    """Initial surrogate ellipsoids for packing (Sec. 2.4): n random centres
    and uniform orientations in a periodic cube sized so that the ellipsoids
    fill `fraction` of it.  Returns (centres [n,3], rotations [n,3,3],
    semi-axes [n,3], side), all float32 (the side exactly representable)."""
    rng = np.random.default_rng(seed)
    vol = 4.0 / 3.0 * math.pi * float(np.prod(semi))
    side = float(np.float32(np.cbrt(n * vol / fraction)))
    centres = (rng.random((n, 3)) * side).astype(np.float32)
    rots = random_rotations(rng, n).astype(np.float32)
    s = np.tile(np.asarray(semi, dtype=np.float32), (n, 1))
    return centres, rots, s, side


def force_bias_pack(rng, n: int, lat: Lattice, wall_clear: float = 2.0,
                    max_iter: int = 400, tol: float = 0.05, step: float = 0.5,
                    max_move: float = 1.5):
    """Random centres and orientations relaxed by the force-bias method.

    Every overlapping pair of cells receives equal and opposite central
    pushes along the line joining their centres, of magnitude given by
    their overlap depth (the pair force of Sec. 2.4, with the depth of the
    deepest surrogate-sphere overlap standing in for the overlap volume).  Orientations stay the
    uniform random draws.  Returns (centres [n,3], rotations [n,3,3],
    residual maximum overlap depth).
    """
    from scipy.spatial import cKDTree

    L = np.array([lat.nx, lat.ny, lat.nz], dtype=np.float64)
    per = np.array([b == PERIODIC for b in lat.bc])
    sph, rad = _surrogate_spheres()
    rest64, _ = _mesh()
    rots = np.stack([random_rotation(rng) for _ in range(n)])
    # per-cell half extent along each axis after rotation (for wall clearance)
    ext = np.abs(np.einsum("cij,vj->cvi", rots, rest64)).max(axis=1)
    lo = np.where(per, 0.0, -0.5 + wall_clear + ext)
    hi = np.where(per, L, L - 0.5 - wall_clear - ext)
    if np.any(hi <= lo):
        raise ValueError("domain too small for wall clearance")
    cen = lo + rng.random((n, 3)) * (hi - lo)
    S = sph.shape[0]
    local = np.einsum("cij,kj->cki", rots, sph)          # [n,S,3]
    box = np.where(per, L, 4.0 * L + 100.0)
    owner = np.repeat(np.arange(n), S)
    maxd = np.inf
    for it in range(max_iter):
        pts = (cen[:, None, :] + local).reshape(-1, 3)
        wrapped = np.where(per, np.mod(pts, L), pts + 2.0 * L + 50.0)
        tree = cKDTree(wrapped, boxsize=box)
        pairs = tree.query_pairs(2 * rad, output_type="ndarray")
        if pairs.size:
            a, b = owner[pairs[:, 0]], owner[pairs[:, 1]]
            keep = a != b
            pairs, a, b = pairs[keep], a[keep], b[keep]
        if pairs.size == 0:
            maxd = 0.0
            break
        d = wrapped[pairs[:, 1]] - wrapped[pairs[:, 0]]
        d = np.where(per, d - L * np.round(d / L), d)
        depth = 2 * rad - np.linalg.norm(d, axis=1)
        maxd = float(depth.max())
        if maxd < tol:
            break
        # aggregate overlap per cell pair, push along the centre line
        key = np.minimum(a, b) * n + np.maximum(a, b)
        uk, inv = np.unique(key, return_inverse=True)
        p = np.zeros(uk.shape[0])
        np.maximum.at(p, inv, depth)
        i, j = uk // n, uk % n
        r = cen[j] - cen[i]
        r = np.where(per, r - L * np.round(r / L), r)
        nr = np.linalg.norm(r, axis=1)
        nr = np.where(nr < 1e-9, 1.0, nr)
        f = (p / nr)[:, None] * r
        disp = np.zeros_like(cen)
        np.add.at(disp, j, f)
        np.add.at(disp, i, -f)
        dn = np.linalg.norm(disp, axis=1, keepdims=True)
        disp = disp * np.minimum(1.0, max_move / np.maximum(dn, 1e-12))
        cen = cen + step * disp
        cen = np.where(per, np.mod(cen, L), np.clip(cen, lo, hi))
    return cen, rots, maxd


# --------------------------------------------------------------------------- workloads
def single_rbc_shear(seed: int = 0) -> Workload:
    """One RBC in a sheared 32^3 box: periodic x/y, z walls moving +-0.01 in x."""
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    lat = Lattice(32, 32, 32, bc=(PERIODIC, PERIODIC, WALL), tau=1.0,
                  wall_u_lo=(-0.01, 0.0, 0.0), wall_u_hi=(0.01, 0.0, 0.0))
    centre = np.array([15.5, 15.5, 15.5]) + rng.uniform(-0.5, 0.5, 3)
    R = small_rotation(rng, 10.0)
    cells = place_cells(rest64, centre[None], R[None], K_REF[None])
    return Workload("single_rbc_shear_32", lat, rest64.astype(np.float32), tri, cells, 500)


def dense_channel(seed: int = 1, n_cells: int = 220) -> Workload:
    """Body-force channel 128x64x64, walls at the y bounds, 220 packed RBCs."""
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    lat = Lattice(128, 64, 64, bc=(PERIODIC, WALL, PERIODIC), tau=1.0, body_force=(1e-5, 0.0, 0.0))
    cen, rots, resid = force_bias_pack(rng, n_cells, lat)
    cells = place_cells(rest64, cen, rots, np.repeat(K_REF[None], n_cells, 0))
    return Workload("dense_channel_128x64x64", lat, rest64.astype(np.float32), tri, cells, 1000,
                    extra={"pack_residual": resid})


def large_suspension(seed: int = 2, n_cells: int = 18600, max_iter: int = 40) -> Workload:
    """Fully periodic 256x256x512 suspension, 18,600 RBCs, body force along z."""
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    lat = Lattice(256, 256, 512, tau=1.0, body_force=(0.0, 0.0, 1e-6))
    cen, rots, resid = force_bias_pack(rng, n_cells, lat, max_iter=max_iter, tol=0.5)
    cells = place_cells(rest64, cen, rots, np.repeat(K_REF[None], n_cells, 0))
    return Workload("large_suspension_256x256x512", lat, rest64.astype(np.float32), tri, cells, 200,
                    extra={"pack_residual": resid})


def batched_calibration(seed: int = 3, n_boxes: int = 256, lo: int = 24, hi: int = 48) -> Workload:
    """Independent periodic cubic boxes, one aligned RBC each, pole traction along x."""
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    sides = rng.integers(lo, hi + 1, size=n_boxes)
    lats, cells = [], []
    for b in range(n_boxes):
        L = int(sides[b])
        lats.append(Lattice(L, L, L, tau=1.0))
        centre = np.full(3, (L - 1) / 2.0) + rng.uniform(-0.5, 0.5, 3)
        F = rng.uniform(0.0, PN200_LU)
        k = log_uniform_k(rng, 1)
        cells.append(place_cells(rest64, centre[None], np.eye(3)[None], k, traction=[[F, 0.0, 0.0]]))
    return Workload("batched_calibration_256", lats, rest64.astype(np.float32), tri, cells, 2000)


def adjoint_boxes(seed: int = 4, n_boxes: int = 64, side: int = 48) -> Workload:
    """Shear + stretch boxes 48^3 with z walls moving +-0.01 in x and seeded targets."""
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    lats, cells, targets = [], [], []
    for b in range(n_boxes):
        tau = rng.uniform(0.8, 1.2)
        lats.append(Lattice(side, side, side, bc=(PERIODIC, PERIODIC, WALL), tau=tau,
                            wall_u_lo=(-0.01, 0.0, 0.0), wall_u_hi=(0.01, 0.0, 0.0)))
        centre = np.full(3, (side - 1) / 2.0) + rng.uniform(-0.5, 0.5, 3)
        F = rng.uniform(0.0, PN200_LU)
        k = log_uniform_k(rng, 1)
        cells.append(place_cells(rest64, centre[None], np.eye(3)[None], k, traction=[[F, 0.0, 0.0]]))
        targets.append([16.0 * rng.uniform(1.0, 1.5), 16.0 * rng.uniform(0.7, 1.0)])
    return Workload("adjoint_64x48", lats, rest64.astype(np.float32), tri, cells, 2000,
                    extra={"targets": np.array(targets), "ckpt_every": 100})


def tiny_periodic(seed: int = 5, n=(24, 20, 16), n_cells: int = 1, walls: int = -1,
                  body=(0.0, 0.0, 0.0), tau: float = 1.0, ibm_kernel: int = 4) -> Workload:
    """Small box for fast parity tests; optional wall axis with moving walls."""
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    bc = [PERIODIC] * 3
    ulo, uhi = [0.0] * 3, [0.0] * 3
    if walls >= 0:
        bc[walls] = WALL
        t = (walls + 1) % 3
        ulo[t], uhi[t] = -0.01, 0.01
    lat = Lattice(*n, bc=tuple(bc), tau=tau, body_force=tuple(body),
                  wall_u_lo=tuple(ulo), wall_u_hi=tuple(uhi), ibm_kernel=ibm_kernel)
    L = np.array(n, dtype=np.float64)
    cen = []
    for c in range(n_cells):
        p = rng.uniform(0, 1, 3) * L
        if walls >= 0:
            p[walls] = (L[walls] - 1) / 2.0 + rng.uniform(-0.5, 0.5)
        cen.append(p)
    rots = np.stack([random_rotation(rng) if walls < 0 else small_rotation(rng, 10.0)
                     for _ in range(n_cells)])
    k = K_REF[None] * 10.0 ** rng.uniform(-0.5, 0.5, (n_cells, 4))
    tr = rng.uniform(-PN200_LU, PN200_LU, (n_cells, 3))
    cells = place_cells(rest64, np.array(cen), rots, k, traction=tr)
    return Workload("tiny", lat, rest64.astype(np.float32), tri, cells, 10)


def small_batch_boxes(seed: int = 0, walls_box: int = 2, kernel: int = 4):
    """Five small boxes of uneven sides for the batched-form parity tests:
    one with z walls moving +-0.01, the others periodic (every other one with
    a body force); one jittered cell per box with log-uniform stiffness and a
    pole traction.  Returns (lattices, rest_pos float32, tri, cells)."""
    sides = [(24, 24, 24), (17, 20, 19), (26, 18, 22), (20, 20, 20), (25, 23, 17)]
    rng = np.random.default_rng(seed)
    rest64, tri = _mesh()
    lats, cells = [], []
    for b, (nx, ny, nz) in enumerate(sides):
        tau = float(rng.uniform(0.8, 1.2))
        if b == walls_box:
            lat = Lattice(nx, ny, nz, bc=(PERIODIC, PERIODIC, WALL), tau=tau, wall_u_lo=(-0.01, 0, 0),
                          wall_u_hi=(0.01, 0, 0), ibm_kernel=kernel)
        else:
            lat = Lattice(nx, ny, nz, tau=tau, body_force=(1e-5 * (b % 2), 0.0, 0.0), ibm_kernel=kernel)
        lats.append(lat)
        centre = np.array([(nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2]) + rng.uniform(-0.5, 0.5, 3)
        R = small_rotation(rng, 8.0)
        c = place_cells(rest64, centre[None], R[None], log_uniform_k(rng, 1),
                        traction=[[rng.uniform(0, PN200_LU), 0.0, 0.0]])
        cells.append(jitter_cells(rng, c, 0.04))
    return lats, rest64.astype(np.float32), tri, cells


# --------------------------------------------------------------------------- random states
def random_shifted_populations(rng, lat: Lattice, scale: float = 1e-3) -> np.ndarray:
    """Random shifted populations g_i = f_i - w_i, float32 [19, nz, ny, nx]."""
    return (scale * rng.standard_normal((19,) + lat.shape)).astype(np.float32)


def jitter_cells(rng, cells: Cells, amp: float = 0.05) -> Cells:
    """Deform cells by a random vertex jitter so every force term is active."""
    off = cells.offsets.astype(np.float64) + amp * rng.standard_normal(cells.offsets.shape)
    return dataclasses.replace(cells, offsets=off.astype(np.float32))


WORKLOADS = {
    "single_rbc_shear_32": single_rbc_shear,
    "dense_channel_128x64x64": dense_channel,
    "large_suspension_256x256x512": large_suspension,
    "batched_calibration_256": batched_calibration,
    "adjoint_64x48": adjoint_boxes,
}
