"""Force-bias packing on the device against the oracle (Sec. 2.4 reading,
oracle/packing.py).

Bars: the overlapping-pair counts are integer work decided in float32, so
they match the oracle's float32 decisions exactly; overlapping volumes
within 1e-5 relative; moved centres within 1e-5 of the largest move plus
the float32 rounding of a centre (2 ulp of the box side).  Multi-iteration
runs are checked one iteration at a time from the device's own state, and
against properties that hold at any size (balanced pushes, wall extents,
bitwise reproducibility, unpacking).
"""
import numpy as np
import pytest

from oracle import packing as P

pytestmark = pytest.mark.gpu


def _rots(rng, n):
    """Uniform random rotations from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)


def _config(rng, n, box, semi, walls=()):
    r = rng.uniform(0, 1, (n, 3)) * np.asarray(box)
    R = _rots(rng, n).astype(np.float32)
    s = np.tile(np.asarray(semi, dtype=np.float32), (n, 1))
    s *= rng.uniform(0.8, 1.0, (n, 1)).astype(np.float32)     # uneven sizes
    e = P.extent(R, s)
    for a in walls:
        r[:, a] = np.clip(r[:, a], 1.5 + e[:, a], box[a] - 1.5 - e[:, a])
    return r.astype(np.float32), R, s


def _domain(box, walls=()):
    per = tuple(a not in walls for a in range(3))
    lo = tuple(1.5 if a in walls else 0.0 for a in range(3))
    hi = tuple(box[a] - 1.5 if a in walls else 0.0 for a in range(3))
    return P.Domain(tuple(box), per, lo, hi)


def _packer(dom, max_semi, eta, max_move, quad):
    from paper_2305_02752_amd import Packer
    return Packer(dom.box, dom.periodic, dom.lo, dom.hi, max_semi=max_semi, eta=eta, max_move=max_move,
                  quad=quad)


def _close(dev, ref, dom, disp_scale):
    d = P.min_image(dev.astype(np.float64) - ref, dom)
    return np.abs(d).max() <= 1e-5 * disp_scale + 2 * 1.2e-7 * max(dom.box)


@pytest.mark.parametrize("walls,quad", [((), 8), ((2,), 8), ((0, 1), 16), ((), 4)])
def test_one_iteration_parity(walls, quad):
    rng = np.random.default_rng(10 + len(walls) + quad)
    box = (56.0, 48.0, 40.0)
    r, R, s = _config(rng, 70, box, (7.0, 6.0, 2.8), walls)
    dom = _domain(box, walls)
    eta, mm = 0.03, 1.0
    pk = _packer(dom, 7.0, eta, mm, quad)
    new, rec = pk.run(r, R, s, 1)
    ref, pairs = P.iterate(r, R, s, dom, eta, mm, quad, np.float32)
    V_ref = sum(p[4] for p in pairs)
    k_ref = sum(1 for p in pairs if p[4] > 0)
    disp = np.abs(P.min_image(ref - r, dom)).max()
    print(walls, quad, "pairs", rec[1], k_ref, "volume", rec[0], V_ref, "max move", disp, flush=True)
    assert rec[1] == k_ref and k_ref > 20
    assert abs(rec[0] - V_ref) <= 1e-5 * V_ref
    assert _close(new, ref, dom, disp)


def test_iteration_chain_and_single_call_agree():
    rng = np.random.default_rng(20)
    box = (48.0, 48.0, 48.0)
    r, R, s = _config(rng, 90, box, (6.5, 6.5, 2.6))
    dom = _domain(box)
    pk = _packer(dom, 6.5, 0.03, 1.0, 8)
    cur = r
    for it in range(6):
        nxt, _ = pk.run(cur, R, s, 1)
        ref, _ = P.iterate(cur, R, s, dom, 0.03, 1.0, 8, np.float32)
        assert _close(nxt, ref, dom, np.abs(P.min_image(ref - cur, dom)).max()), it
        cur = nxt
    once, rec = pk.run(r, R, s, 6)
    assert np.array_equal(once, cur)                 # one call of 6 = 6 calls of 1, bit for bit
    again, rec2 = pk.run(r, R, s, 6)
    assert np.array_equal(once, again) and rec == rec2


def test_balanced_pushes_and_walls():
    rng = np.random.default_rng(21)
    box = (60.0, 44.0, 52.0)
    r, R, s = _config(rng, 120, box, (7.0, 7.0, 2.8))
    dom = _domain(box)
    # periodic, no move clamp: the pair pushes cancel exactly in sum
    pk = _packer(dom, 7.0, 1e-3, 1e6, 8)
    new, rec = pk.run(r, R, s, 1)
    d = P.min_image(new.astype(np.float64) - r, dom)
    assert rec[1] > 30
    assert np.abs(d.sum(axis=0)).max() <= len(r) * 2 * 1.2e-7 * max(box)
    r, R, s = _config(rng, 120, box, (7.0, 7.0, 2.8), walls=(1,))
    dom = _domain(box, walls=(1,))
    pk = _packer(dom, 7.0, 0.05, 2.0, 8)
    new, _ = pk.run(r, R, s, 10)
    e = P.extent(R, s)
    tol = 1e-5
    assert np.all(new[:, 1] - e[:, 1] >= 1.5 - tol) and np.all(new[:, 1] + e[:, 1] <= box[1] - 1.5 + tol)


def test_few_bins_per_axis():
    """A periodic side of two bins and a wall axis of one bin: neighbour bins
    must not be visited twice."""
    rng = np.random.default_rng(22)
    box = (30.0, 60.0, 16.0)
    r, R, s = _config(rng, 40, box, (6.0, 6.0, 2.4), walls=(2,))
    dom = _domain(box, walls=(2,))
    pk = _packer(dom, 6.0, 0.03, 1.0, 8)
    new, rec = pk.run(r, R, s, 1)
    ref, pairs = P.iterate(r, R, s, dom, 0.03, 1.0, 8, np.float32)
    assert rec[1] == sum(1 for p in pairs if p[4] > 0) > 10
    assert _close(new, ref, dom, np.abs(P.min_image(ref - r, dom)).max())


def test_dense_unpacking_and_refusals():
    rng = np.random.default_rng(23)
    L = 96.0
    semi = (8.5, 8.5, 3.2)
    n = int(0.35 * L ** 3 / P.volume(semi))
    r, R, s = _config(rng, n, (L, L, L), semi)
    dom = _domain((L, L, L))
    pk = _packer(dom, 8.5, 0.03, 1.0, 8)
    _, rec = pk.run(r, R, s, 80)
    print("cells", n, "overlap", rec, flush=True)
    assert rec[2] < 0.01 * rec[0] and rec[3] < 0.2 * rec[1]
    from paper_2305_02752_amd.hemo import HemoError
    with pytest.raises(HemoError, match="HC_ERR_ARG"):
        _packer(dom, 8.5, 0.03, 1.0, 5).run(r, R, s, 1)
    with pytest.raises(HemoError, match="HC_ERR_ARG"):
        _packer(_domain((30.0, L, L)), 8.5, 0.03, 1.0, 8).run(r, R, s, 1)   # side < 4 max_semi
    with pytest.raises(HemoError, match="HC_ERR_ARG"):
        _packer(dom, 8.0, 0.03, 1.0, 8).run(r, R, s, 1)                     # a semi-axis > max_semi
    out, rec0 = pk.run(r[:0], R[:0], s[:0], 3)                             # no ellipsoids
    assert out.shape == (0, 3) and rec0 == (0.0, 0.0, 0.0, 0.0)


def test_large_sampled_parity():
    """A million-ellipsoid-scale run is too large for the brute-force
    oracle; one iteration at 200k ellipsoids is checked on sampled ellipsoids,
    each against the oracle run on it and every ellipsoid within reach."""
    rng = np.random.default_rng(24)
    semi = np.array([8.5, 8.5, 3.2])
    n = 200_000
    L = float(np.float32(np.cbrt(n * P.volume(semi) / 0.35)))   # a side float32 holds exactly
    box = (L, L, L)
    r, R, s = _config(rng, n, box, semi)
    dom = _domain(box)
    pk = _packer(dom, 8.5, 0.03, 1.0, 8)
    new, rec = pk.run(r, R, s, 1)
    assert rec[1] > 0.5 * n
    reach = 2 * 8.5
    for i in rng.choice(n, 40, replace=False):
        d = P.min_image(r.astype(np.float64) - r[i].astype(np.float64), dom)
        near = np.nonzero((np.abs(d) < reach + 1).all(axis=1))[0]
        sub = np.r_[[i], near[near != i]]
        ref, _ = P.iterate(r[sub], R[sub], s[sub], dom, 0.03, 1.0, 8, np.float32)
        assert _close(new[i:i + 1], ref[:1], dom, np.abs(P.min_image(ref[:1] - r[i:i + 1], dom)).max() + 1e-3)


def test_pack_then_place_cells_on_device():
    """Packed ellipsoids become cells without leaving the device: the
    placement matches the host placement of the same centres and rotations
    (float32 offsets within 4e-6, a few ulp), and the packed suspension steps."""
    import torch

    from paper_2305_02752_amd import Simulation
    from workloads import rbc_mesh
    from workloads.configs import RBC_SURROGATE, Lattice, place_cells

    rng = np.random.default_rng(25)
    lat = Lattice(64, 48, 48, tau=1.0, body_force=(1e-6, 0.0, 0.0))
    box = (64.0, 48.0, 48.0)
    n = int(0.25 * 64 * 48 * 48 / P.volume(RBC_SURROGATE))
    r, R, s = _config(rng, n, box, RBC_SURROGATE)
    s[:] = np.asarray(RBC_SURROGATE, dtype=np.float32)
    pk = _packer(_domain(box), max(RBC_SURROGATE), 0.03, 1.0, 8)
    dev = torch.device("cuda:0")
    tc = torch.tensor(r, device=dev)
    tr = torch.tensor(R.reshape(-1, 9), device=dev)
    ts = torch.tensor(s, device=dev)
    rec = pk.run_device(tc, tr, ts, 60)
    assert rec[3] < 0.2 * rec[1]
    rest64, tri = rbc_mesh()
    k = np.tile([1.5e-4, 1e-5, 5e-2, 1e-2], (n, 1))
    sim = Simulation(lat, rest64.astype(np.float32), tri, max_cells=n)
    sim.place_cells(tc, tr, k)
    o, off, _ = sim.read_vertices()
    ref = place_cells(rest64.astype(np.float32).astype(np.float64), tc.cpu().numpy().astype(np.float64),
                      R.astype(np.float64), k)
    assert np.array_equal(o, ref.origin)
    assert np.abs(off - ref.offsets).max() <= 4e-6
    sim.init_equilibrium()
    sim.step(5)
    sim.sync()
    o2, off2, _ = sim.read_vertices()
    assert np.isfinite(off2).all()
