"""Pins of the membrane oracle (Sec. 2.3 force decomposition).

Checks: mesh topology and the paper's RBC dimensions, the area and volume
against an independent convex-hull routine, zero force at rest, rigid-motion
invariance, zero net force and torque, and force = -grad(energy) by central
finite differences for every term separately.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial import ConvexHull
from scipy.spatial.transform import Rotation

from oracle import membrane as M
from workloads import rbc_mesh, sphere_mesh

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
UM_PER_LU = 0.5


@pytest.fixture(scope="module")
def cell():
    V, T = rbc_mesh()
    topo = M.Topology(T, V.shape[0])
    return V, T, topo, M.RestState(V, topo)


def _deformed(cell, seed=0, amp=0.03):
    V = cell[0]
    rng = np.random.default_rng(seed)
    return V + amp * rng.standard_normal(V.shape)


def test_mesh_topology(cell):
    V, T, topo, _ = cell
    assert V.shape == (642, 3) and T.shape == (1280, 3)
    assert len(topo.edges) == 1920 and len(topo.hinges) == 1920
    assert V.shape[0] - len(topo.edges) + T.shape[0] == 2          # Euler characteristic
    # every directed edge appears once: consistent orientation of a closed surface
    d = {(int(a), int(b)) for t in T for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    assert len(d) == 3 * T.shape[0] and all((b, a) in d for a, b in d)


def test_rbc_dimensions_match_paper(cell):
    V = cell[0]
    dia = np.ptp(V[:, 0]) * UM_PER_LU
    thick = np.ptp(V[:, 2]) * UM_PER_LU
    g = GOLD
    assert g["rbc_diameter_um"]["min"] <= dia <= g["rbc_diameter_um"]["max"]
    assert g["rbc_thickness_um"]["min"] <= thick <= g["rbc_thickness_um"]["max"]
    # biconcave: the centre is thinner than the rim
    centre = np.abs(V[np.hypot(V[:, 0], V[:, 1]) < 1.0, 2]).max()
    assert 2 * centre < 0.5 * np.ptp(V[:, 2])


def test_area_volume_against_convex_hull():
    V, T = sphere_mesh(3, 4.0)
    A, Vol = M.area_volume(V[None], T)
    hull = ConvexHull(V)
    assert abs(A[0] - hull.area) < 1e-10 * hull.area
    assert abs(Vol[0] - hull.volume) < 1e-10 * hull.volume
    # both below the smooth sphere's, within the icosphere's discretisation error
    assert 0.98 * 4 * np.pi * 16 < A[0] < 4 * np.pi * 16
    assert 0.97 * 4 / 3 * np.pi * 64 < Vol[0] < 4 / 3 * np.pi * 64


def test_rbc_volume_positive_and_translation_free(cell):
    V, T, _, rest = cell
    assert rest.V0 > 0 and rest.A0 > 0
    A2, V2 = M.area_volume(V[None] + np.array([123.4, -56.7, 89.0]), T)
    assert abs(V2[0] - rest.V0) < 1e-9 and abs(A2[0] - rest.A0) < 1e-10


def test_dihedral_convex_positive_and_exact_under_hinge_rotation(cell):
    """theta > 0 on a convex surface; rotating one wing rigidly about the
    hinge edge by delta changes theta by exactly delta."""
    Vs, Ts = sphere_mesh(3, 4.0)
    ts = M.Topology(Ts, Vs.shape[0])
    assert (M.dihedral(Vs[None], ts.hinges) > 0).all()
    V, _, topo, _ = cell
    X = _deformed(cell, 5)
    for h in (0, 17, 900, 1919):
        i, j, k, l = topo.hinges[h]
        th = M.dihedral(X, topo.hinges[h:h + 1])[0]
        e = (X[j] - X[i]) / np.linalg.norm(X[j] - X[i])
        for delta in (0.01, -0.02):
            R = Rotation.from_rotvec(delta * e).as_matrix()
            Y = X.copy()
            Y[l] = X[i] + R @ (X[l] - X[i])
            th2 = M.dihedral(Y, topo.hinges[h:h + 1])[0]
            assert abs(abs(th2 - th) - abs(delta)) < 1e-12
            # folding the second wing about +e (right-handed) opens a convex fold
            assert np.sign(th2 - th) == np.sign(delta)


def test_zero_force_at_rest(cell):
    V, _, topo, rest = cell
    k = np.array([[1.5e-4, 1e-5, 5e-2, 1e-2]])
    F = M.forces(V[None], k, topo, rest)
    assert np.abs(F).max() < 1e-14 * k.max()


def test_rigid_motion_invariance(cell):
    _, _, topo, rest = cell
    X = _deformed(cell)
    k = np.array([[1.0, 1.0, 1.0, 1.0]])
    F = M.forces(X[None], k, topo, rest)[0]
    for seed in range(3):
        R = Rotation.random(random_state=seed).as_matrix()
        c = np.random.default_rng(seed).uniform(-50, 50, 3)
        F2 = M.forces((X @ R.T + c)[None], k, topo, rest)[0]
        assert np.abs(F2 - F @ R.T).max() < 1e-9 * np.abs(F).max()


def test_zero_net_force_and_torque(cell):
    _, _, topo, rest = cell
    X = _deformed(cell, 1)
    for term in ("link", "bend", "area", "volume"):
        F = M.forces(X[None], np.ones((1, 4)), topo, rest, terms=(term,))[0]
        s = np.abs(F).max()
        assert np.abs(F.sum(0)).max() < 1e-12 * s * 642
        assert np.abs(np.cross(X, F).sum(0)).max() < 1e-11 * s * 642 * 10


@pytest.mark.parametrize("term,idx", [("link", 0), ("bend", 1), ("area", 2), ("volume", 3)])
def test_force_is_minus_energy_gradient(cell, term, idx):
    _, _, topo, rest = cell
    X = _deformed(cell, 2)[None]
    k = np.zeros((1, 4))
    k[0, idx] = 1.0
    F = M.forces(X, k, topo, rest, terms=(term,))
    h = 1e-6
    scale = np.abs(F).max()
    rng = np.random.default_rng(idx)
    for v in rng.choice(642, 6, replace=False):
        for d in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[0, v, d] += h
            Xm[0, v, d] -= h
            g = (M.energy(Xp, k, topo, rest) - M.energy(Xm, k, topo, rest))[0] / (2 * h)
            assert abs(-g - F[0, v, d]) < 1e-6 * scale


def test_nonlinear_link_stiffens(cell):
    """Link response is linear at small strain and stiffer at large strain (Sec. 2.3)."""
    s = np.array([1e-4, 0.5, 1.5, 2.5])
    g = M._g(s, M.TAU_LINK)
    assert abs(g[0] / s[0] - (1 + 1 / M.TAU_LINK ** 2)) < 1e-6
    assert np.all(np.diff(g / s) > 0)


def test_traction_poles(cell):
    V, _, topo, rest = cell
    assert len(rest.p_plus) == len(rest.p_minus) == 32
    assert V[rest.p_plus, 0].min() >= np.sort(V[:, 0])[-32] - 1e-12
    assert V[rest.p_minus, 0].max() <= np.sort(V[:, 0])[31] + 1e-12
    F = M.forces(V[None], np.zeros((1, 4)), topo, rest, traction=np.array([[3.2, 0.0, 0.0]]))
    assert np.abs(F[0].sum(0)).max() < 1e-14
    assert abs(F[0, rest.p_plus, 0].sum() - 3.2) < 1e-14
