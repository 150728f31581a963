"""Pins of the oracle's loss and of its two gradients.

The oracle has two gradients of the loss: central differences of the full
FP64 run, and the complex-step method (forward-mode differentiation of the
same run on complex numbers, exact to rounding).  These tests show the
differences are converged (step sizes a decade apart agree), that the loss
seed (dL/dX at the extreme vertices) is the derivative of the loss, that
the complex step reproduces a closed-form first-step derivative, and that
the two gradients agree.
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


# ---------------------------------------------------------------------------
# Complex-step gradient (the oracle's second, difference-free gradient)


def _jittered_setup(seed=3):
    """A deformed cell (vertex jitter 0.05 lu), so that every force term is
    active and finite differences are accurate."""
    from oracle import membrane, step  # noqa: F401
    rng = np.random.default_rng(seed)
    rest64, tri = rbc_mesh()
    lat = Lattice(20, 20, 20, bc=(0, 0, 1), tau=0.9, wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    cells = place_cells(rest64, np.array([[9.6, 9.3, 9.5]]), np.eye(3)[None], K_REF[None],
                        traction=[[3e-3, 0, 0]])
    X0 = cells.positions64()[0] + 0.05 * rng.standard_normal((rest64.shape[0], 3))
    return lat, rest64.astype(np.float32), tri, X0, cells.traction[0]


def test_complex_step_matches_closed_form_first_step():
    """One step from rest (rho = 1, u = 0): the vertex velocity is the
    interpolated half of the spread membrane force, which is linear in each
    stiffness, so dX1/dk_j = interp(spread(F_j) / 2) with F_j the force at
    unit k_j (others zero), and dL/dk_j follows from the four extreme
    vertices; X1 does not depend on tau (dL/dtau = 0)."""
    from oracle import ibm, lattice, membrane, step
    lat, rest, tri, X0, tr = _jittered_setup()
    targets = (19.0, 14.0)
    g = oadj.cs_gradient(lat, rest, tri, X0, K_REF, tr, lat.tau, 1, targets)
    m = step.make_model(lat, rest.astype(np.float64), tri, K_REF[None], tr[None])
    f0 = lattice.init_equilibrium(lat.shape)
    _, X1, _ = step.step(m, f0, X0[None])
    X1 = X1[0]
    ia, ib, ic, id_ = oadj.extremes(X1)
    da, dt = oadj.diameters(X1)
    dims = (lat.nx, lat.ny, lat.nz)
    want = np.zeros(5)
    for j in range(4):
        kj = np.zeros((1, 4))
        kj[0, j] = 1.0
        Fj = membrane.forces(X0[None], kj, m.topo, m.rest, None)[0]
        u = ibm.spread(X0, Fj, dims, lat.bc, 4) / 2.0
        dX = ibm.interpolate(u, X0, dims, lat.bc, (0, 0, 0), (0, 0, 0), 4)
        want[j] = 2 * (da - targets[0]) * (dX[ia, 0] - dX[ib, 0]) + 2 * (dt - targets[1]) * (dX[ic, 1] - dX[id_, 1])
    assert g[4] == 0.0
    assert np.abs(g[:4] - want[:4]).max() <= 1e-10 * np.abs(want[:4]).max()
    assert np.abs(want[:4]).min() > 0


def test_complex_step_matches_fd():
    lat, rest, tri, X0, tr = _jittered_setup()
    targets = (19.0, 14.0)
    n = 12
    g_cs = oadj.cs_gradient(lat, rest, tri, X0, K_REF, tr, lat.tau, n, targets)
    g_fd = oadj.fd_gradient(lat, rest, tri, X0, K_REF, tr, lat.tau, n, targets, eps=1e-4)
    p = np.concatenate([K_REF, [lat.tau]])
    # normwise (the metric of the adjoint parity bar)
    assert np.linalg.norm(p * (g_cs - g_fd)) <= 1e-7 * np.linalg.norm(p * g_fd)
    # componentwise within the accuracy of central differences: a perturbed
    # loss of about 10 changes by only ~1e-9 for the small components, so
    # rounding of the loss limits them to a few 1e-6
    assert np.all(np.abs(p * (g_cs - g_fd)) <= 1e-5 * np.abs(p * g_fd))


def test_stored_full_box_gradients_agree():
    """The stored full-size gradients (48^3, 2000 steps) by the oracle's two
    independent methods: central differences and the complex step."""
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    fd = np.load(os.path.join(here, "adjoint_full_boxes_fd.npz"))
    cs = np.load(os.path.join(here, "adjoint_full_boxes_cs.npz"))
    assert (fd["boxes"] == cs["boxes"]).all() and fd["steps"] == cs["steps"] == 2000
    for b in range(len(fd["boxes"])):
        p = fd["params"][b]
        pf, pc = p * fd["fd_grad"][b], p * cs["cs_grad"][b]
        assert np.linalg.norm(pf - pc) <= 1e-6 * np.linalg.norm(pc)
