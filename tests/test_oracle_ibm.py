"""Pins of the immersed-boundary oracle (Sec. 2.3 coupling).

Closed-form properties of Peskin's 4-point function and exact identities of
spreading and interpolation with the same kernel.
"""
import numpy as np
import pytest

from oracle import ibm


def test_phi4_closed_form_values():
    assert ibm.phi4(0.0) == 0.5                      # (3 + 1)/8
    assert abs(ibm.phi4(1.0) - 0.25) < 1e-16         # (3 - 2 + 1)/8 = (5 - 2 - 1)/8
    assert ibm.phi4(2.0) == 0.0 and ibm.phi4(2.5) == 0.0
    assert abs(ibm.phi4(0.5) - (2 + np.sqrt(2)) / 8) < 1e-15
    # continuity across r = 1 and r = 2
    assert abs(ibm.phi4(1 - 1e-12) - ibm.phi4(1 + 1e-12)) < 1e-9
    assert abs(ibm.phi4(2 - 1e-12)) < 1e-5


@pytest.mark.parametrize("kernel", [4, 2])
def test_kernel_moments(kernel):
    """Partition of unity and zero first moment for every offset; for phi4
    also sum phi^2 = 3/8 (Peskin's conditions)."""
    phi = ibm.phi4 if kernel == 4 else ibm.phi2
    r = np.linspace(0.0, 1.0, 1001)[:-1]
    ks = np.arange(-1, 3) if kernel == 4 else np.arange(0, 2)
    w = np.stack([phi(r - k) for k in ks])
    assert np.abs(w.sum(0) - 1).max() < 1e-14
    assert np.abs((w * (r[None] - ks[:, None])).sum(0)).max() < 1e-14
    if kernel == 4:
        assert np.abs((w ** 2).sum(0) - 3 / 8).max() < 1e-14
        even = w[0::2].sum(0)
        assert np.abs(even - 0.5).max() < 1e-14    # sum over even nodes = sum over odd nodes


@pytest.mark.parametrize("kernel", [4, 2])
def test_spread_conserves_total_force(kernel):
    rng = np.random.default_rng(0)
    dims = (9, 7, 11)
    X = rng.uniform(0, 1, (50, 3)) * np.array(dims) * 1.3 - 2.0   # includes wrap-around
    Fv = rng.standard_normal((50, 3))
    F = ibm.spread(X, Fv, dims, (0, 0, 0), kernel)
    assert np.allclose(F.reshape(3, -1).sum(1), Fv.sum(0), atol=1e-12)


@pytest.mark.parametrize("bc", [(0, 0, 0), (0, 1, 0), (0, 0, 1)])
def test_transpose_identity(bc):
    """sum_x F(x).u(x) = sum_v F_v.U_v for any fields (walls at rest)."""
    rng = np.random.default_rng(1)
    dims = (8, 10, 9)
    X = rng.uniform(0.2, 0.8, (40, 3)) * np.array(dims)
    Fv = rng.standard_normal((40, 3))
    u = rng.standard_normal((3, dims[2], dims[1], dims[0]))
    F = ibm.spread(X, Fv, dims, bc)
    U = ibm.interpolate(u, X, dims, bc, (0, 0, 0), (0, 0, 0))
    assert abs((F * u).sum() - (Fv * U).sum()) < 1e-11


def test_linear_field_interpolates_exactly():
    rng = np.random.default_rng(2)
    dims = (16, 16, 16)
    z, y, x = np.meshgrid(*[np.arange(n, dtype=float) for n in dims[::-1]], indexing="ij")
    a = rng.standard_normal(3)
    B = rng.standard_normal((3, 3))
    u = np.stack([a[d] + B[d, 0] * x + B[d, 1] * y + B[d, 2] * z for d in range(3)])
    X = rng.uniform(3, 12, (30, 3))
    U = ibm.interpolate(u, X, dims, (0, 0, 0), (0, 0, 0), (0, 0, 0))
    assert np.allclose(U, a + X @ B.T, atol=1e-12)


def test_wall_nodes_read_wall_velocity():
    """A vertex touching a wall with fluid at rest sees a blend of the wall speed."""
    dims = (8, 8, 8)
    u = np.zeros((3, 8, 8, 8))
    X = np.array([[4.3, 4.6, 0.25]])
    U = ibm.interpolate(u, X, dims, (0, 0, 1), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    assert np.abs(U).max() == 0
    U = ibm.interpolate(u, X, dims, (0, 0, 1), (1.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    # the node below the wall (z = -1) carries weight phi4(1.25)
    assert abs(U[0, 0] - ibm.phi4(1.25)) < 1e-15
