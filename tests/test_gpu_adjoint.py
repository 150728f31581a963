"""Adjoint form: device reverse sweep vs FP64 central differences of the oracle.

Loss: (D_A - D_A*)^2 + (D_T - D_T*)^2 of one cell after n coupled steps in a
sheared box with a pole traction.  Parameters p = (k_link, k_bend, k_area,
k_volume, tau), also with an interior viscosity ratio (tau then also sets
the interior relaxation time).  Bar: p . dL/dp normwise within 1e-4 of the
FP64 finite-difference gradient; bit-identical gradients for any checkpoint
interval.
"""
import numpy as np
import pytest

from oracle import adjoint as oadj
from workloads import rbc_mesh
from workloads.configs import K_REF, Lattice, place_cells, small_rotation

from gpu_common import make_sim

pytestmark = pytest.mark.gpu


def _box(seed=0, side=20, walls=True):
    rng = np.random.default_rng(seed)
    rest64, tri = rbc_mesh()
    if walls:
        lat = Lattice(side, side, side, bc=(0, 0, 1), tau=float(rng.uniform(0.8, 1.2)),
                      wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    else:
        lat = Lattice(side, side, side, tau=float(rng.uniform(0.8, 1.2)))
    k = K_REF * 10.0 ** rng.uniform(-0.5, 0.5, 4)
    centre = np.full(3, (side - 1) / 2.0) + rng.uniform(-0.5, 0.5, 3)
    cells = place_cells(rest64, centre[None], small_rotation(rng, 5.0)[None], k[None],
                        traction=[[3e-3, 0.0, 0.0]])
    targets = np.array([16.0 * 1.2, 16.0 * 0.9])
    return lat, rest64.astype(np.float32), tri, cells, targets


def _device_grad(lat, rest, tri, cells, targets, n, ck, ratio=1.0):
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest, tri=tri, cells=cells), cells)
    sim.init_equilibrium()
    sim.set_interior_viscosity(ratio)
    sim.adj_bind(n, ck)
    loss = sim.adj_forward(targets)
    g = sim.adj_backward()
    return loss[0], g[0], sim


@pytest.mark.parametrize("walls,ratio", [(True, 1.0), (False, 1.0), (True, 5.0)])
def test_adjoint_matches_fd(walls, ratio):
    lat, rest, tri, cells, targets = _box(1 if walls else 2, walls=walls)
    n = 40
    loss, g, _ = _device_grad(lat, rest, tri, cells, targets, n, 10, ratio)
    X0 = cells.positions64()[0]
    k = cells.k[0].astype(np.float64)
    L_ref, _ = oadj.run_loss(lat, rest, tri, X0, k, cells.traction[0], lat.tau, n, targets,
                             interior_ratio=ratio)
    g_fd = oadj.fd_gradient(lat, rest, tri, X0, k, cells.traction[0], lat.tau, n, targets, eps=1e-4,
                            interior_ratio=ratio)
    p = np.concatenate([k, [lat.tau]])
    pg, pf = p * g, p * g_fd
    comp = np.abs(pg - pf) / np.maximum(np.abs(pf), 1e-30)
    norm = np.linalg.norm(pg - pf) / np.linalg.norm(pf)
    print(f"ratio {ratio}: loss {loss:.8f} vs {L_ref:.8f}; p.g {pg}; fd {pf}; comp {comp}; norm {norm:.2e}",
          flush=True)
    assert abs(loss - L_ref) <= 1e-5 * abs(L_ref)
    assert norm <= 1e-4
    # the oracle's second, difference-free gradient (complex step)
    g_cs = oadj.cs_gradient(lat, rest, tri, X0, k, cells.traction[0], lat.tau, n, targets,
                            interior_ratio=ratio)
    pc = p * g_cs
    norm_cs = np.linalg.norm(pg - pc) / np.linalg.norm(pc)
    print(f"  vs complex step: {pc}; norm {norm_cs:.2e}", flush=True)
    assert norm_cs <= 1e-4


def test_adjoint_backward_refers_to_latest_forward():
    """A parameter change between hc_adj_forward and hc_adj_backward
    discards the forward (its reverse sweep would recompute under other
    parameters): the backward is refused until the next forward."""
    from paper_2305_02752_amd import HemoError
    lat, rest, tri, cells, targets = _box(4)
    loss, g, sim = _device_grad(lat, rest, tri, cells, targets, 12, 4)
    sim.set_params(k=cells.k * 1.1, tau=lat.tau)
    with pytest.raises(HemoError) as e:
        sim.adj_backward()
    assert e.value.code == 2   # HC_ERR_STATE
    sim.set_params(k=cells.k, tau=lat.tau)
    with pytest.raises(HemoError):
        sim.adj_backward()


def test_coupled_step_fn_two_forwards_then_backward():
    """Two applies on one runner, then backward of the first: refused (the
    contexts hold the second forward's checkpoints); the second's backward
    is the second's gradient."""
    import torch
    from paper_2305_02752_amd.autograd import AdjointBoxes, CoupledStepFn
    boxes = [_box(20 + b) for b in range(2)]
    runner = AdjointBoxes([b[0] for b in boxes], boxes[0][1], boxes[0][2], [b[3] for b in boxes],
                          [b[4] for b in boxes], n_steps=12, ckpt_every=4)
    p0 = np.array([np.concatenate([b[3].k[0], [b[0].tau]]) for b in boxes])
    pa = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    pb = torch.tensor(p0 * np.array([1.2, 1.0, 1.0, 1.0, 1.0]), dtype=torch.float64, requires_grad=True)
    la = CoupledStepFn.apply(pa, runner)
    lb = CoupledStepFn.apply(pb, runner)
    with pytest.raises(RuntimeError):
        la.sum().backward()
    lb.sum().backward()
    ref = AdjointBoxes([b[0] for b in boxes], boxes[0][1], boxes[0][2], [b[3] for b in boxes],
                       [b[4] for b in boxes], n_steps=12, ckpt_every=4)
    ref.forward(pb.detach().numpy())
    assert np.array_equal(pb.grad.numpy(), ref.backward())


@pytest.mark.parametrize("ratio", [1.0, 5.0])
def test_adjoint_checkpoint_interval_is_exact(ratio):
    lat, rest, tri, cells, targets = _box(3)
    _, g1, _ = _device_grad(lat, rest, tri, cells, targets, 24, 24, ratio)
    _, g2, _ = _device_grad(lat, rest, tri, cells, targets, 24, 5, ratio)
    assert np.array_equal(g1, g2)


def test_coupled_step_fn_autograd():
    import torch
    from paper_2305_02752_amd.autograd import AdjointBoxes, CoupledStepFn
    boxes = [_box(10 + b) for b in range(3)]
    runner = AdjointBoxes([b[0] for b in boxes], boxes[0][1], boxes[0][2], [b[3] for b in boxes],
                          [b[4] for b in boxes], n_steps=20, ckpt_every=5)
    p0 = np.array([np.concatenate([b[3].k[0], [b[0].tau]]) for b in boxes])
    params = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    loss = CoupledStepFn.apply(params, runner)
    (loss * torch.tensor([1.0, 2.0, -0.5], dtype=torch.float64)).sum().backward()
    for b in range(3):
        _, g, _ = _device_grad(boxes[b][0], boxes[b][1], boxes[b][2], boxes[b][3], boxes[b][4], 20, 5)
        w = [1.0, 2.0, -0.5][b]
        # the runner's boxes share one shape: batched reverse sweep (same
        # arithmetic as the single-box one, compiled a second time)
        assert np.linalg.norm(params.grad[b].numpy() - w * g) <= 1e-6 * np.linalg.norm(w * g)


def test_adjoint_with_per_cell_interior_ratios():
    """Two cells with different interior viscosity ratios (two classes):
    dL/dtau, which reaches the interior sites of each class through its own
    tau_k, and dL/dk_link of each cell against FP64 central differences of
    the summed loss."""
    import dataclasses

    from oracle import lattice as olat, step as ostep
    rng = np.random.default_rng(60)
    rest64, tri = rbc_mesh()
    lat = Lattice(40, 24, 24, bc=(0, 0, 1), tau=0.95, wall_u_lo=(-0.01, 0, 0), wall_u_hi=(0.01, 0, 0))
    k = K_REF * 10.0 ** rng.uniform(-0.3, 0.3, (2, 4))
    cells = place_cells(rest64, np.array([[10.6, 11.7, 11.4], [29.3, 12.2, 11.6]]),
                        np.stack([small_rotation(rng, 5.0) for _ in range(2)]), k,
                        traction=[[3e-3, 0.0, 0.0], [-2e-3, 0.0, 0.0]])
    targets = np.array([[16.0 * 1.2, 16.0 * 0.9], [16.0 * 1.1, 16.0 * 0.95]])
    ratios = np.array([3.0, 6.0])
    n = 24
    from types import SimpleNamespace
    sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest64.astype(np.float32), tri=tri, cells=cells),
                   cells)
    sim.init_equilibrium()
    sim.set_cell_viscosity(ratios)
    sim.adj_bind(n, 8)
    loss = sim.adj_forward(targets.reshape(-1))
    g = sim.adj_backward()

    X0 = cells.positions64()
    kk = cells.k.astype(np.float64)
    tr = cells.traction.astype(np.float64)

    def total_loss(tau, kmat):
        m = ostep.make_model(dataclasses.replace(lat, tau=float(tau)), rest64, tri, kmat, tr,
                             interior_ratio=ratios)
        _, X = ostep.run(m, olat.init_equilibrium(lat.shape), X0, n)
        return sum(oadj.loss_of(X[c], targets[c]) for c in range(2))

    assert abs(loss.sum() - total_loss(lat.tau, kk)) <= 1e-5 * abs(loss.sum())
    h = 1e-4 * lat.tau
    fd_tau = (total_loss(lat.tau + h, kk) - total_loss(lat.tau - h, kk)) / (2 * h)
    fd_k = []
    for c in range(2):
        hk = 1e-4 * kk[c, 0]
        kp, km = kk.copy(), kk.copy()
        kp[c, 0] += hk
        km[c, 0] -= hk
        fd_k.append((total_loss(lat.tau, kp) - total_loss(lat.tau, km)) / (2 * hk))
    pg = np.array([lat.tau * g[0, 4], kk[0, 0] * g[0, 0], kk[1, 0] * g[1, 0]])
    pf = np.array([lat.tau * fd_tau, kk[0, 0] * fd_k[0], kk[1, 0] * fd_k[1]])
    norm = np.linalg.norm(pg - pf) / np.linalg.norm(pf)
    print("p.g", pg, "fd", pf, "norm", norm, flush=True)
    assert np.allclose(g[:, 4], g[0, 4])       # tau is shared
    assert norm <= 1e-4


def test_adjoint_full_size_properties():
    # one box of the adjoint workload at its full configuration (48^3,
    # moving walls, pole traction, 2000 steps, checkpoint every 100), as the
    # benchmark runs it.  The FP64 oracle cannot take 2000 steps of 48^3 in
    # test time, so the checks are properties that hold at any size: the
    # checkpointed forward is the plain run bit for bit, its loss is the loss
    # of its final vertices, and the gradient is finite and does not depend
    # on the checkpoint interval.
    from paper_2305_02752_amd import Simulation
    from workloads import adjoint_boxes
    w = adjoint_boxes(seed=4, n_boxes=1)   # box 0 of the 64-box workload
    n, ck = w.steps, w.extra["ckpt_every"]
    c, tg = w.cells[0], w.extra["targets"][0]

    def make():
        sim = Simulation(w.lattice[0], w.rest_pos, w.tri, max_cells=1)
        sim.set_cells(c.origin, c.offsets, c.k, c.traction)
        sim.init_equilibrium()
        return sim

    plain = make()
    plain.step(n)
    plain.sync()
    a = make()
    a.adj_bind(n, ck)
    loss = a.adj_forward(tg)[0]
    assert np.array_equal(a.read_populations(), plain.read_populations())
    o, off = a.read_vertices()[:2]
    assert np.array_equal(off, plain.read_vertices()[1])
    L_host = oadj.loss_of(o[0][None, :] + off[0].astype(np.float64), tg)
    g1 = a.adj_backward()[0]
    b = make()
    b.adj_bind(n, 40)
    assert b.adj_forward(tg)[0] == loss
    g2 = b.adj_backward()[0]
    print(f"loss {loss:.8f} (host {L_host:.8f}), grad {g1}", flush=True)
    assert abs(loss - L_host) <= 1e-5 * abs(L_host)
    assert np.all(np.isfinite(g1)) and np.any(g1 != 0.0)
    assert np.array_equal(g1, g2)


def test_adjoint_forward_leaves_the_last_step_fields():
    """The adjoint forward writes the force and (u, rho) fields at its last
    step only; with field output on, reading them afterwards gives what a
    plain run of the same steps gives: bit for bit from hc_adj_forward (the
    same kernels), within a few FP32 roundings from the batched form."""
    from types import SimpleNamespace

    from paper_2305_02752_amd import Simulation
    n = 40
    boxes = [_box(seed=s_) for s_ in (3, 4)]

    def make(b):
        lat, rest, tri, cells, _ = b
        sim = make_sim(SimpleNamespace(lattice=lat, rest_pos=rest, tri=tri, cells=cells), cells)
        sim.init_equilibrium()
        return sim

    plain = []
    for b in boxes:
        sim = make(b)
        sim.step(n)
        sim.sync()
        plain.append((sim.read_macro(), sim.read_force_field()))
        sim.close()
    sim = make(boxes[0])
    sim.adj_bind(n, 15)
    sim.adj_forward(boxes[0][4])
    (rho, u), F = sim.read_macro(), sim.read_force_field()
    sim.close()
    assert np.array_equal(rho, plain[0][0][0]) and np.array_equal(u, plain[0][0][1])
    assert np.array_equal(F, plain[0][1])
    sims = [make(b) for b in boxes]
    for s_ in sims:
        s_.adj_bind(n, 15)
    Simulation.adj_multi_forward(sims, np.stack([b[4] for b in boxes])[:, None, :])
    for k, s_ in enumerate(sims):
        (rho, u), F = s_.read_macro(), s_.read_force_field()
        (rho0, u0), F0 = plain[k]
        assert np.abs(rho - rho0).max() <= 1e-6 * np.abs(rho0).max()
        assert np.abs(u - u0).max() <= 1e-6 * np.abs(u0).max()
        assert np.abs(F - F0).max() <= 1e-6 * np.abs(F0).max()
        s_.close()


def test_multi_box_adjoint_equals_single_box():
    """hc_adj_multi_forward / _backward over three boxes of the adjoint
    workload's shape (48^3, sheared; 240 steps, checkpoint every 50, so the
    last segment is short) give each box the loss, state and gradient of its
    own hc_adj_forward / hc_adj_backward: the same arithmetic, in kernels
    compiled a second time (the compiler may fuse a multiply-add differently),
    so equal to within a few FP32 roundings."""
    from types import SimpleNamespace

    from paper_2305_02752_amd import Simulation
    from workloads import adjoint_boxes
    w = adjoint_boxes()
    n, ck, boxes = 240, 50, (0, 1, 2)

    def make(b):
        c = w.cells[b]
        sim = make_sim(SimpleNamespace(lattice=w.lattice[b], rest_pos=w.rest_pos, tri=w.tri, cells=c), c)
        sim.init_equilibrium()
        sim.adj_bind(n, ck)
        return sim

    single = []
    for b in boxes:
        sim = make(b)
        loss = sim.adj_forward(w.extra["targets"][b])
        g = sim.adj_backward()
        single.append((loss, g, sim.read_populations(), sim.read_vertices()[1]))
        sim.close()
    sims = [make(b) for b in boxes]
    loss = Simulation.adj_multi_forward(sims, w.extra["targets"][list(boxes)])
    g = Simulation.adj_multi_backward(sims)
    for k, b in enumerate(boxes):
        print(f"box {b}: loss {loss[k][0]:.10f} vs {single[k][0][0]:.10f}; grad {g[k][0]}", flush=True)
        assert np.allclose(loss[k], single[k][0], rtol=1e-7, atol=0)
        assert np.linalg.norm(g[k] - single[k][1]) <= 1e-6 * np.linalg.norm(single[k][1])
        pops = single[k][2]
        assert np.abs(sims[k].read_populations() - pops).max() <= 1e-6 * np.abs(pops).max()
        off = single[k][3]
        assert np.abs(sims[k].read_vertices()[1] - off).max() <= 1e-6
    # a second forward/backward from the new state works the same way
    loss2 = Simulation.adj_multi_forward(sims, w.extra["targets"][list(boxes)])
    assert np.all(np.isfinite(loss2)) and np.all(np.isfinite(Simulation.adj_multi_backward(sims)))
    for s in sims:
        s.close()
