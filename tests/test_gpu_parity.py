"""Device path (libhemo through the C ABI) against the FP64 oracle.

Tolerances: one step <= 1e-5 max relative error per field (populations
compared shifted, g = f - w; vertex displacement and forces relative to
their field maxima); many steps <= 1e-3.  Integer binning bit-exact.
"""
import numpy as np
import pytest

from oracle import binning, lattice, membrane, step
from workloads import jitter_cells, random_shifted_populations, single_rbc_shear, tiny_periodic
from workloads.configs import Lattice, place_cells, K_REF

from gpu_common import make_sim, oracle_model, oracle_state, relerr

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5
TOL_LONG = 1e-3

CASES = {
    # name: (workload kwargs, jitter)
    "periodic_1cell": dict(seed=5, n=(24, 20, 16), n_cells=1),
    "periodic_3cells_body": dict(seed=6, n=(32, 24, 20), n_cells=3, body=(2e-5, -1e-5, 5e-6)),
    "wall_z_moving": dict(seed=7, n=(24, 20, 16), n_cells=1, walls=2),
    "wall_y_moving": dict(seed=8, n=(28, 24, 20), n_cells=1, walls=1, body=(1e-5, 0, 0)),
    "wall_x_tau07": dict(seed=9, n=(24, 26, 28), n_cells=1, walls=0, tau=0.7),
    "phi2_kernel": dict(seed=10, n=(24, 20, 16), n_cells=2, ibm_kernel=2),
    # last tile 1 node wide on x and z: a stencil window meets 3 tiles per axis
    "ragged_tiles_33_25": dict(seed=11, n=(33, 20, 25), n_cells=3),
}


def _one_step(name):
    w = tiny_periodic(**CASES[name])
    rng = np.random.default_rng(100)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    sim.step(1)
    sim.sync()
    g1 = sim.read_populations()
    rho, u = sim.read_macro()
    F = sim.read_force_field()
    o1, off1, fv = sim.read_vertices()
    U = sim.read_vertex_velocity()
    m = oracle_model(w, cells)
    f0, X0 = oracle_state(g0, cells)
    f1r, X1r, info = step.step(m, f0, X0)
    X1 = o1[:, None, :].astype(np.float64) + off1.astype(np.float64)
    _check_positions(X1, X1r, off1, info["U"])
    return dict(g=(g1, lattice.shifted(f1r)), rho=(rho, info["rho"]), u=(u, info["u"]),
                F=(F, info["F"]), Fv=(fv, info["Fv"]), U=(U, info["U"]))


def _check_positions(Xg, Xr, off, Ur):
    """Positions are stored as float32 offsets, so X^{n+1} = X^n + U carries
    the rounding of the offset (half an ulp, <= 6e-8 |offset|) on top of the
    error of U itself."""
    bound = 6e-8 * np.abs(off).max() + TOL_STEP * np.abs(Ur).max()
    assert np.abs(Xg - Xr).max() <= bound, (np.abs(Xg - Xr).max(), bound)


@pytest.mark.parametrize("name", list(CASES))
def test_one_step_parity(name):
    res = _one_step(name)
    errs = {k: relerr(a, b) for k, (a, b) in res.items()}
    print(name, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= TOL_STEP, (k, e)


def test_one_step_parity_dense_channel():
    # the dense channel suspension at its full size (128 x 64 x 64, walls at
    # the y bounds, body force, 220 cells), one step from random shifted
    # populations and jittered cells, every field against the oracle
    from workloads import dense_channel
    w = dense_channel()
    rng = np.random.default_rng(101)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    sim.step(1)
    sim.sync()
    rho, u = sim.read_macro()
    o1, off1, fv = sim.read_vertices()
    m = oracle_model(w, cells)
    f0, X0 = oracle_state(g0, cells)
    f1r, X1r, info = step.step(m, f0, X0)
    _check_positions(o1[:, None, :].astype(np.float64) + off1.astype(np.float64), X1r, off1, info["U"])
    errs = {"g": relerr(sim.read_populations(), lattice.shifted(f1r)), "rho": relerr(rho, info["rho"]),
            "u": relerr(u, info["u"]), "F": relerr(sim.read_force_field(), info["F"]),
            "Fv": relerr(fv, info["Fv"]), "U": relerr(sim.read_vertex_velocity(), info["U"])}
    print("dense channel", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= TOL_STEP, (k, e)


def test_zero_cells_fluid_only():
    lat = Lattice(20, 12, 16, bc=(0, 1, 0), tau=0.8, body_force=(1e-5, 0, 0))
    from workloads import rbc_mesh
    rest, tri = rbc_mesh()
    from paper_2305_02752_amd import Simulation
    sim = Simulation(lat, rest.astype(np.float32), tri, max_cells=0)
    rng = np.random.default_rng(3)
    g0 = random_shifted_populations(rng, lat, 1e-3)
    sim.write_populations(g0)
    sim.step(3)
    sim.sync()
    f = lattice.unshift(g0)
    F = np.zeros((3,) + lat.shape)
    F[0] = 1e-5
    for _ in range(3):
        f, _, _ = lattice.lbm_step(f, F, 0.8, bc=(0, 1, 0))
    assert relerr(sim.read_populations(), lattice.shifted(f)) <= TOL_STEP


def test_cell_across_periodic_corner():
    w = tiny_periodic(seed=12, n=(24, 20, 16), n_cells=1)
    rest64 = w.rest_pos.astype(np.float64)
    from workloads.configs import random_rotation
    rng = np.random.default_rng(4)
    cells = place_cells(rest64, np.array([[0.3, 19.6, 0.2]]), random_rotation(rng)[None],
                        K_REF[None], traction=[[1e-3, 2e-3, -1e-3]])
    cells = jitter_cells(rng, cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    sim = make_sim(w, cells)
    sim.write_populations(g0)
    sim.step(1)
    sim.sync()
    m = oracle_model(w, cells)
    f0, X0 = oracle_state(g0, cells)
    f1, X1, info = step.step(m, f0, X0)
    o, off, fv = sim.read_vertices()
    assert relerr(sim.read_populations(), lattice.shifted(f1)) <= TOL_STEP
    assert relerr(fv, info["Fv"]) <= TOL_STEP
    assert relerr(sim.read_vertex_velocity(), info["U"]) <= TOL_STEP
    _check_positions(o[:, None, :] + off.astype(np.float64), X1, off, info["U"])


def test_membrane_area_volume_fp64():
    w = tiny_periodic(seed=13, n=(40, 40, 40), n_cells=4)
    rng = np.random.default_rng(5)
    cells = jitter_cells(rng, w.cells, 0.1)
    sim = make_sim(w, cells)
    fv, A, V = sim.compute_forces()
    m = oracle_model(w, cells)
    X = cells.positions64()
    Ar, Vr = membrane.area_volume(X, m.topo.tri)
    assert np.abs(A - Ar).max() / Ar.max() < 1e-12
    assert np.abs(V - Vr).max() / Vr.max() < 1e-12
    Fr = membrane.forces(X, m.k, m.topo, m.rest, m.traction)
    assert relerr(fv, Fr) <= TOL_STEP


@pytest.mark.parametrize("kernel,walls", [(4, -1), (4, 1), (2, 2), (2, -1)])
def test_binning_bit_exact(kernel, walls):
    n = (40, 33, 24) if walls != 2 else (40, 33, 26)
    w = tiny_periodic(seed=14, n=n, n_cells=4 if walls < 0 else 1, walls=walls, ibm_kernel=kernel)
    rng = np.random.default_rng(6)
    cells = jitter_cells(rng, w.cells, 0.05)
    sim = make_sim(w, cells)
    sim.step(2)
    sim.sync()
    owner, tptr, touch, cptr, clist = sim.read_bins()
    o, off, _ = sim.read_vertices()
    dims, bc = (w.lattice.nx, w.lattice.ny, w.lattice.nz), w.lattice.bc
    ow, _, _, cptr_r, clist_r = binning.bins(o, off, dims, bc)
    tptr_r, touch_r = binning.touch_lists(o, off, dims, bc, kernel)
    assert np.array_equal(owner, ow)
    assert np.array_equal(cptr, cptr_r) and np.array_equal(clist, clist_r)
    assert np.array_equal(tptr, tptr_r) and np.array_equal(touch, touch_r)


@pytest.mark.parametrize("scale,n", [(2.8, (72, 64, 56)), (1.0, (24, 24, 24))])
def test_binning_bit_exact_cell_sizes(scale, n):
    """A cell reaching more than 6 tiles per axis (its pairs are ranked in
    the LDS hash), and a cell reaching every tile of a 3-tile lattice (the
    direct table over the whole cyclic axis)."""
    from workloads import rbc_mesh
    from workloads.configs import random_rotation
    rng = np.random.default_rng(31)
    rest64, tri = rbc_mesh()
    lat = Lattice(*n)
    rot = np.eye(3) if scale > 2 else random_rotation(rng)   # the large cell's diameter along x
    cells = place_cells(scale * rest64, np.array(n, dtype=float)[None] / 2 + rng.uniform(-1, 1, (1, 3)),
                        rot[None], K_REF[None])
    cells = jitter_cells(rng, cells, 0.05)
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=(scale * rest64).astype(np.float32), tri=tri,
                                   cells=cells), cells)
    sim.step(2)
    sim.sync()
    owner, tptr, touch, cptr, clist = sim.read_bins()
    o, off, _ = sim.read_vertices()
    dims = (lat.nx, lat.ny, lat.nz)
    ow, _, _, cptr_r, clist_r = binning.bins(o, off, dims, lat.bc)
    tptr_r, touch_r = binning.touch_lists(o, off, dims, lat.bc, 4)
    assert np.array_equal(owner, ow)
    assert np.array_equal(cptr, cptr_r) and np.array_equal(clist, clist_r)
    assert np.array_equal(tptr, tptr_r) and np.array_equal(touch, touch_r)
    if scale > 2:
        x = o[0, 0] + off[0, :, 0]
        assert x.max() - x.min() > 5 * 8   # beyond the direct table's 6 tiles


def test_deterministic_bitwise():
    w = tiny_periodic(seed=15, n=(32, 24, 24), n_cells=3, body=(1e-5, 0, 0))
    rng = np.random.default_rng(7)
    cells = jitter_cells(rng, w.cells, 0.05)
    g0 = random_shifted_populations(rng, w.lattice, 1e-3)
    outs = []
    for _ in range(2):
        sim = make_sim(w, cells)
        sim.write_populations(g0)
        sim.step(20)
        sim.sync()
        outs.append((sim.read_populations(), sim.read_vertices()[1]))
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_checkpoint_resume_bitwise():
    w = tiny_periodic(seed=16, n=(24, 24, 24), n_cells=2)
    rng = np.random.default_rng(8)
    cells = jitter_cells(rng, w.cells, 0.05)
    sim = make_sim(w, cells)
    sim.step(10)
    ck = sim.checkpoint_save()
    sim.step(15)
    sim.sync()
    ref = (sim.read_populations(), sim.read_vertices()[1])
    sim2 = make_sim(w, cells)
    sim2.checkpoint_restore(ck)
    assert sim2.steps_taken() == 10
    sim2.step(15)
    sim2.sync()
    assert np.array_equal(sim2.read_populations(), ref[0])
    assert np.array_equal(sim2.read_vertices()[1], ref[1])


def test_nonfinite_flag_surfaces():
    from paper_2305_02752_amd import HemoError
    w = tiny_periodic(seed=17, n=(24, 24, 24), n_cells=1)
    sim = make_sim(w)
    o, off, _ = sim.read_vertices()
    off = off.copy()
    off[0, 5, 1] = np.nan
    sim.write_vertices(o, off)
    sim.step(1)
    with pytest.raises(HemoError) as e:
        sim.sync()
    assert e.value.code == 5
    sim.sync()          # flag cleared


def test_multistep_single_rbc_shear_500():
    """Single RBC in shear (32^3, moving z walls), 500 steps <= 1e-3."""
    w = single_rbc_shear()
    sim = make_sim(w)
    sim.init_equilibrium()
    sim.step(w.steps)
    sim.sync()
    m = oracle_model(w, w.cells)
    f = lattice.init_equilibrium(w.lattice.shape)
    X0 = w.cells.positions64()
    f, X = step.run(m, f, X0, w.steps)
    o, off, _ = sim.read_vertices()
    Xg = o[:, None, :] + off.astype(np.float64)
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    e_x = relerr(Xg - X0, X - X0)
    print("500 steps: pops", e_g, "displacement", e_x, flush=True)
    assert e_g <= TOL_LONG and e_x <= TOL_LONG


def test_multistep_1000_tiny():
    w = tiny_periodic(seed=18, n=(24, 20, 16), n_cells=1, walls=2)
    rng = np.random.default_rng(9)
    cells = jitter_cells(rng, w.cells, 0.02)
    sim = make_sim(w, cells)
    sim.init_equilibrium()
    sim.step(1000)
    sim.sync()
    m = oracle_model(w, cells)
    f = lattice.init_equilibrium(w.lattice.shape)
    X0 = cells.positions64()
    f, X = step.run(m, f, X0, 1000)
    o, off, _ = sim.read_vertices()
    e_g = relerr(sim.read_populations(), lattice.shifted(f))
    e_x = relerr(o[:, None, :] + off.astype(np.float64) - X0, X - X0)
    print("1000 steps: pops", e_g, "displacement", e_x, flush=True)
    assert e_g <= TOL_LONG and e_x <= TOL_LONG


def test_cell_carried_past_recentring():
    """A cell carried ~20 lu by a uniform stream (0.1 lu/step, 200 steps) in a
    periodic 40 x 24 x 24 box, with a pole traction deforming it: its origin
    is re-centred on the way (the bounding-box centre may not stray more than
    8 lu from the integer origin), origin + offsets stay within 1e-3 of the
    oracle's positions (relative to the largest displacement), and the
    binning of the re-centred (origin, offsets) is bit-exact."""
    from types import SimpleNamespace

    from workloads import rbc_mesh
    from workloads.configs import small_rotation
    rng = np.random.default_rng(17)
    rest64, tri = rbc_mesh()
    lat = Lattice(40, 24, 24, tau=1.0)
    cells = place_cells(rest64, np.array([[10.3, 11.7, 12.2]]), small_rotation(rng, 10.0)[None], K_REF[None],
                        traction=[[2e-3, 0.0, 0.0]])
    cells = jitter_cells(rng, cells, 0.05)
    w = SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri, cells=cells)
    sim = make_sim(w, cells)
    u0 = (0.1, 0.0, 0.0)
    sim.init_equilibrium(u0=u0)
    n = 200
    sim.step(n)
    sim.sync()
    o, off, _ = sim.read_vertices()
    owner, tptr, touch, cptr, clist = sim.read_bins()
    sim.close()
    m = oracle_model(w, cells)
    X0 = cells.positions64()
    _, X = step.run(m, lattice.init_equilibrium(lat.shape, u0=u0), X0, n)
    Xg = o[:, None, :].astype(np.float64) + off.astype(np.float64)
    e_x = relerr(Xg - X0, X - X0)
    mid = 0.5 * (off.min(axis=1) + off.max(axis=1))
    print(f"origin {cells.origin[0]} -> {o[0]}, box centre offset {mid[0]}, displacement max "
          f"{np.abs(X - X0).max():.2f} lu, error {e_x:.2e}", flush=True)
    assert o[0, 0] - cells.origin[0, 0] >= 8          # re-centred at least once along x
    assert np.abs(mid).max() <= 8.0 + 0.1 * 1.5      # at most one move past the threshold
    assert np.abs(X - X0).max() > 16.0
    assert e_x <= TOL_LONG
    dims, bc = (lat.nx, lat.ny, lat.nz), lat.bc
    ow, _, _, cptr_r, clist_r = binning.bins(o, off, dims, bc)
    tptr_r, touch_r = binning.touch_lists(o, off, dims, bc, lat.ibm_kernel)
    assert np.array_equal(owner, ow)
    assert np.array_equal(cptr, cptr_r) and np.array_equal(clist, clist_r)
    assert np.array_equal(tptr, tptr_r) and np.array_equal(touch, touch_r)


def test_membrane_forces_independent_of_workgroup_size():
    """One jittered cell's membrane forces and FP64 area/volume are bit for
    bit the same whether the per-cell kernel runs it with 1024 threads (1
    cell), 512 (65 cells) or 256 (1025 cells), and as hc_compute_forces
    (256 threads): the area/volume sums do not depend on the work-group."""
    from types import SimpleNamespace

    from workloads import rbc_mesh
    from workloads.configs import random_rotation
    rng = np.random.default_rng(23)
    rest64, tri = rbc_mesh()
    lat = Lattice(128, 128, 128)
    n_max = 1025
    cen = rng.uniform(8, 120, (n_max, 3))
    rots = np.stack([random_rotation(rng) for _ in range(n_max)])
    k = K_REF[None] * 10.0 ** rng.uniform(-0.5, 0.5, (n_max, 4))
    cells = jitter_cells(rng, place_cells(rest64, cen, rots, k, traction=rng.uniform(-1e-3, 1e-3, (n_max, 3))), 0.05)
    out = []
    for n in (1, 65, 1025):
        sub = SimpleNamespace(origin=cells.origin[:n], offsets=cells.offsets[:n], k=cells.k[:n],
                              traction=cells.traction[:n], n=n)
        sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri, cells=sub), sub)
        fv2, area, volume = sim.compute_forces()   # 256 threads, initial positions
        fv2 = fv2[0].copy()
        sim.step(1)                                # the first step's forces, same positions
        sim.sync()
        _, _, fv = sim.read_vertices()
        out.append((fv[0].copy(), fv2, area[0], volume[0]))
        sim.close()
    for fv, fv2, a, v in out:
        assert np.array_equal(fv, out[0][0]) and np.array_equal(fv2, out[0][0])
        assert a == out[0][2] and v == out[0][3]


def test_crowded_tiles_need_a_larger_list_capacity():
    """30 overlapping cells in a 24^3 box: the fullest tile list exceeds the
    default capacity, so hc_set_cells refuses them and names the capacity it
    needs; with that capacity (lists past 512 entries, staged in chunks, and
    the force bound on the capacity's coarser grid) one step matches the
    oracle field by field."""
    from types import SimpleNamespace

    from paper_2305_02752_amd import Simulation
    from paper_2305_02752_amd.hemo import HemoError
    from workloads import rbc_mesh
    from workloads.configs import random_rotation
    rng = np.random.default_rng(29)
    rest64, tri = rbc_mesh()
    lat = Lattice(24, 24, 24, bc=(0, 0, 1), tau=0.9, wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    n = 30
    cen = 11.5 + rng.uniform(-2.5, 2.5, (n, 3))
    rots = np.stack([random_rotation(rng) for _ in range(n)])
    k = K_REF[None] * 10.0 ** rng.uniform(-0.5, 0.5, (n, 4))
    cells = jitter_cells(rng, place_cells(rest64, cen, rots, k, traction=rng.uniform(-2e-3, 2e-3, (n, 3))), 0.05)
    rest = rest64.astype(np.float32)
    sim = Simulation(lat, rest, tri, max_cells=n)
    with pytest.raises(HemoError) as err:
        sim.set_cells(cells.origin, cells.offsets, cells.k, cells.traction)
    need = int(str(err.value).split("needs ")[1].split(" ")[0])
    print("fullest list", need, flush=True)
    assert need > 2048
    sim.close()
    cap = 1 << int(np.ceil(np.log2(need)))
    sim = Simulation(lat, rest, tri, max_cells=n, list_capacity=cap)
    sim.set_cells(cells.origin, cells.offsets, cells.k, cells.traction)
    assert sim.densest_tile() == (need, cap)
    rng2 = np.random.default_rng(3)
    g0 = random_shifted_populations(rng2, lat, 1e-3)
    sim.write_populations(g0)
    sim.step(1)
    sim.sync()
    rho, u = sim.read_macro()
    _, _, fv = sim.read_vertices()
    w = SimpleNamespace(lattice=lat, rest_pos=rest, tri=tri)
    m = oracle_model(w, cells)
    f0, X0 = oracle_state(g0, cells)
    f1, X1, info = step.step(m, f0, X0)
    errs = {"g": relerr(sim.read_populations(), lattice.shifted(f1)), "u": relerr(u, info["u"]),
            "F": relerr(sim.read_force_field(), info["F"]), "Fv": relerr(fv, info["Fv"]),
            "U": relerr(sim.read_vertex_velocity(), info["U"])}
    print({kk: f"{v:.2e}" for kk, v in errs.items()}, flush=True)
    sim.close()
    for kk, e in errs.items():
        assert e <= TOL_STEP, (kk, e)



def test_list_overflow_recovers_from_a_checkpoint():
    """A tile list that overflows during a run (the cells, set spread out in
    a 48^3 box with the fullest list at 1,173 entries, are written into one
    crowded spot whose fullest list holds 8,179) is reported by hc_sync;
    the run then continues from its last checkpoint in a context with a
    larger list capacity and stays within the one-step tolerance of a run
    that had that capacity from the start (the capacity sets the force
    bound's grid, so the two differ only in fixed-point rounding)."""
    from paper_2305_02752_amd import Simulation
    from paper_2305_02752_amd.hemo import HemoError
    from workloads import rbc_mesh
    from workloads.configs import random_rotation
    rng = np.random.default_rng(31)
    rest64, tri = rbc_mesh()
    rest = rest64.astype(np.float32)
    lat = Lattice(48, 48, 48, tau=0.9, body_force=(1e-5, 0.0, 0.0))
    n = 30
    rots = np.stack([random_rotation(rng) for _ in range(n)])
    k = K_REF[None] * 10.0 ** rng.uniform(-0.5, 0.5, (n, 4))
    spread = place_cells(rest64, rng.uniform(6, 42, (n, 3)), rots, k)
    crowded = place_cells(rest64, 19.5 + rng.uniform(-2.5, 2.5, (n, 3)), rots, k)
    g0 = random_shifted_populations(np.random.default_rng(5), lat, 1e-3)

    def start(cap):
        sim = Simulation(lat, rest, tri, max_cells=n, list_capacity=cap)
        sim.set_cells(spread.origin, spread.offsets, spread.k, None)
        return sim

    sim = start(None)   # the default capacity, 2048
    sim.write_populations(g0)
    sim.step(2)
    sim.sync()
    ck = sim.checkpoint_save()
    sim.write_vertices(crowded.origin, crowded.offsets)
    sim.step(1)
    with pytest.raises(HemoError, match="exceeded its capacity"):
        sim.sync()
    sim.close()
    cap = 1 << 14
    rec = start(cap)
    rec.checkpoint_restore(ck)
    ref = start(cap)
    ref.write_populations(g0)
    ref.step(2)
    ref.sync()
    for s_ in (rec, ref):
        s_.write_vertices(crowded.origin, crowded.offsets)
        s_.step(3)
        s_.sync()
    assert rec.densest_tile()[1] == cap
    o1, x1, _ = rec.read_vertices()
    o2, x2, _ = ref.read_vertices()
    errs = {"g": relerr(rec.read_populations(), ref.read_populations()),
            "X": relerr((o1[:, None, :] + x1.astype(np.float64)) - crowded.positions64(),
                        (o2[:, None, :] + x2.astype(np.float64)) - crowded.positions64())}
    print({kk: f"{v:.2e}" for kk, v in errs.items()}, flush=True)
    rec.close()
    ref.close()
    assert np.array_equal(o1, o2)
    for kk, e in errs.items():
        assert e <= TOL_STEP, (kk, e)