"""Full-size check: the large suspension (256 x 256 x 512, 18,600 cells) in
the launch configuration the benchmark times, one step from random shifted
populations and jittered cells, checked on sampled outputs that the FP64
oracle can compute one by one:

  * membrane forces of sampled cells (oracle.membrane on the input positions);
  * post-collision populations of sampled nodes, read where streaming put
    them: the node's force density is spread by oracle.ibm from the oracle
    forces of the nearby cells on a local 16^3 patch centred on the node;
  * interpolated velocities of sampled vertices, from oracle moments on the
    vertex's 4^3 stencil nodes;
  * owner tiles of all 11.9M vertices, bit-exact.
"""
import numpy as np
import pytest

from oracle import binning, ibm, lattice, membrane, step
from workloads import jitter_cells, large_suspension

from gpu_common import relerr

pytestmark = pytest.mark.gpu

PATCH = 16
C0 = PATCH // 2


@pytest.fixture(scope="module")
def run():
    w = large_suspension()
    rng = np.random.default_rng(123)
    cells = jitter_cells(rng, w.cells, 0.03)
    lat = w.lattice
    g0 = (1e-3 * rng.standard_normal((19,) + lat.shape, dtype=np.float32)).astype(np.float32)
    from paper_2305_02752_amd import Simulation
    sim = Simulation(lat, w.rest_pos, w.tri, max_cells=cells.n)
    sim.set_cells(cells.origin, cells.offsets, cells.k, None)
    sim.write_populations(g0)
    sim.step(1)
    sim.sync()
    g1 = sim.read_populations()
    o1, off1, fv = sim.read_vertices()
    vel = sim.read_vertex_velocity()
    owner_gpu, *_ = sim.read_bins()
    sim.close()
    model = step.make_model(lat, w.rest_pos.astype(np.float64), w.tri, cells.k)
    return dict(w=w, cells=cells, g0=g0, g1=g1, fv=fv, vel=vel, owner=owner_gpu, model=model,
                o1=o1, off1=off1, rng=np.random.default_rng(7))


class Neighbourhood:
    """Cells whose vertices lie near a point (periodic minimum image)."""

    def __init__(self, cells, dims):
        self.X = cells.positions64()
        self.dims = np.array(dims, dtype=np.float64)
        self.centre = self.X.mean(axis=1)

    def cells_near(self, p, reach):
        d = self.centre - p
        d -= self.dims * np.round(d / self.dims)
        return np.nonzero(np.all(np.abs(d) < reach + 14.0, axis=1))[0]

    def local(self, cids, p):
        """Vertex positions of cells cids relative to p + patch centre."""
        X = self.X[cids]
        d = X - p
        d -= self.dims * np.round(d / self.dims)
        return d + C0


def _forces(run, cids, cache):
    m = run["model"]
    out = []
    for c in cids:
        if c not in cache:
            X = run["cells"].positions64()[c:c + 1]
            cache[c] = membrane.forces(X, m.k[c:c + 1], m.topo, m.rest)[0]
        out.append(cache[c])
    return np.stack(out) if out else np.zeros((0, 642, 3))


def _local_force(run, nb, cache, p):
    """Force density on a 16^3 patch centred on node p.  Only vertices within
    6 nodes of p are spread, so the patch's own wrap-around cannot alias any
    contribution onto the nodes within 3 of the centre that the tests read."""
    cids = nb.cells_near(p, 4.0)
    Xl = nb.local(cids, p).reshape(-1, 3)
    Fv = _forces(run, cids, cache).reshape(-1, 3)
    keep = np.all(np.abs(Xl - C0) < 6.0, axis=1)
    F = ibm.spread(Xl[keep], Fv[keep], (PATCH,) * 3, (0, 0, 0), 4)
    g = np.array(run["w"].lattice.body_force)
    return F + g[:, None, None, None]


def test_fullsize_membrane_forces(run):
    m = run["model"]
    idx = run["rng"].choice(run["cells"].n, 16, replace=False)
    X = run["cells"].positions64()[idx]
    ref = membrane.forces(X, m.k[idx], m.topo, m.rest)
    assert relerr(run["fv"][idx], ref) <= 1e-5


def test_fullsize_owner_tiles_bit_exact(run):
    """Owner tiles of every vertex, on the device's own positions after the step."""
    lat = run["w"].lattice
    ref = binning.vertex_owner(run["o1"], run["off1"], (lat.nx, lat.ny, lat.nz), lat.bc).ravel()
    assert np.array_equal(run["owner"], ref)


def test_fullsize_collide_stream_samples(run):
    w, lat = run["w"], run["w"].lattice
    nb = Neighbourhood(run["cells"], (lat.nx, lat.ny, lat.nz))
    cache = {}
    nx, ny, nz = lat.nx, lat.ny, lat.nz
    f0 = run["g0"]
    got, ref = [], []
    for _ in range(48):
        x, y, z = (int(run["rng"].integers(0, n)) for n in (nx, ny, nz))
        F = _local_force(run, nb, cache, np.array([x, y, z], dtype=np.float64))[:, C0, C0, C0]
        f = lattice.unshift(f0[:, z, y, x][:, None])
        rho, u = lattice.moments(f, F[:, None])
        post = lattice.collide(f, rho, u, F[:, None], lat.tau)[:, 0]
        for i in range(19):
            ex, ey, ez = lattice.E[i]
            got.append(run["g1"][i, (z + ez) % nz, (y + ey) % ny, (x + ex) % nx])
            ref.append(post[i] - lattice.W[i])
    assert relerr(np.array(got), np.array(ref)) <= 1e-5


def test_fullsize_interpolation_samples(run):
    w, lat = run["w"], run["w"].lattice
    nb = Neighbourhood(run["cells"], (lat.nx, lat.ny, lat.nz))
    cache = {}
    X = run["cells"].positions64()
    dims = np.array([lat.nx, lat.ny, lat.nz])
    got, ref = [], []
    for _ in range(24):
        c = int(run["rng"].integers(0, run["cells"].n))
        v = int(run["rng"].integers(0, 642))
        p = np.floor(X[c, v])
        F = _local_force(run, nb, cache, p)
        # populations on the patch (global nodes p - C0 .. p + C0 - 1, wrapped)
        idx = [(np.arange(PATCH) - C0 + int(p[d])) % dims[d] for d in range(3)]
        f = lattice.unshift(run["g0"][:, idx[2]][:, :, idx[1]][:, :, :, idx[0]])
        _, u = lattice.moments(f, F)
        U = ibm.interpolate(u, (X[c, v] - p + C0)[None], (PATCH,) * 3, (0, 0, 0), (0, 0, 0), (0, 0, 0))
        got.append(run["vel"][c, v])
        ref.append(U[0])
    assert relerr(np.array(got), np.array(ref)) <= 1e-5
