"""The configurations at their own lengths, against stored oracle results.

The oracle cannot run these in test time, so `tests/golden/make_goldens.py`
(which calls only the FP64 oracle and the seeded input generators) stored
its results once; the device runs the same inputs here.  Bars: fields and
displacements within 1e-3 (max relative, against the full field's maximum)
after 1000 steps; adjoint gradients p . dL/dp within 1e-4 (normwise) of the
oracle's finite-difference and complex-step gradients at the adjoint
workload's full size (48^3, 2000 steps, checkpoint every 100).
"""
import os

import numpy as np
import pytest

from gpu_common import make_sim

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_LONG = 1e-3
TOL_GRAD = 1e-4


def _adjoint_device(b):
    from types import SimpleNamespace

    from workloads import adjoint_boxes
    w = adjoint_boxes()
    c = w.cells[b]
    sim = make_sim(SimpleNamespace(lattice=w.lattice[b], rest_pos=w.rest_pos, tri=w.tri, cells=c), c)
    sim.init_equilibrium()
    sim.adj_bind(w.steps, w.extra["ckpt_every"])
    loss = sim.adj_forward(w.extra["targets"][b])[0]
    g = sim.adj_backward()[0]
    sim.close()
    return loss, g


@pytest.mark.parametrize("which", [0, 1])
def test_adjoint_full_box_gradient(which):
    fd = np.load(os.path.join(GOLDEN, "adjoint_full_boxes_fd.npz"))
    cs = np.load(os.path.join(GOLDEN, "adjoint_full_boxes_cs.npz"))
    b = int(fd["boxes"][which])
    assert fd["steps"] == 2000 and fd["ckpt_every"] == 100 and int(cs["boxes"][which]) == b
    assert fd["extremes_same"][which].all()     # each difference quotient on one smooth branch
    loss, g = _adjoint_device(b)
    p = fd["params"][which]
    pg = p * g
    for name, ref in (("fd", fd["fd_grad"][which]), ("cs", cs["cs_grad"][which])):
        pr = p * ref
        norm = np.linalg.norm(pg - pr) / np.linalg.norm(pr)
        print(f"box {b}: loss {loss:.8f} vs {fd['loss'][which]:.8f}; p.g {pg}; {name} {pr}; norm {norm:.2e}",
              flush=True)
        assert norm <= TOL_GRAD, name
    assert abs(loss - fd["loss"][which]) <= TOL_GRAD * abs(fd["loss"][which])


def test_dense_channel_1000_steps():
    # 128 x 64 x 64, walls at the y bounds, body force along x, 220 cells,
    # 1000 steps from rest on the device against the stored FP64 run
    from workloads import dense_channel
    path = os.path.join(GOLDEN, "dense_channel_1000.npz")
    if not os.path.exists(path):
        pytest.skip("stored run missing: python tests/golden/make_goldens.py dense_channel")
    ref = np.load(path)
    w = dense_channel()
    assert int(ref["steps"]) == w.steps == 1000
    sim = make_sim(w)
    sim.init_equilibrium()
    sim.step(w.steps)
    sim.sync()
    g = sim.read_populations().reshape(19, -1)
    o, off, _ = sim.read_vertices()
    sim.close()
    s = int(ref["vertex_stride"])
    disp = (o[:, None, :].astype(np.float64) + off.astype(np.float64) - w.cells.positions64())[:, ::s, :]
    e_x = np.abs(disp - ref["displacement"]).max() / float(ref["displacement_max"])
    e_g = np.abs(g[:, ref["sites"]] - ref["populations"]).max() / float(ref["populations_max"])
    print(f"dense channel 1000 steps: displacement {e_x:.2e} (max {float(ref['displacement_max']):.3f} lu), "
          f"populations {e_g:.2e}", flush=True)
    assert e_x <= TOL_LONG and e_g <= TOL_LONG


def test_batch_1000_steps():
    # the five batched-form boxes (one walled, two with a body force), one
    # persistent launch per run call, 1000 steps from rest
    from paper_2305_02752_amd import Batch
    from workloads.configs import small_batch_boxes
    ref = np.load(os.path.join(GOLDEN, "batch_boxes_1000.npz"))
    lats, rest, tri, cells = small_batch_boxes(int(ref["seed"]))
    bt = Batch(lats, rest, tri)
    bt.set_cells(np.concatenate([c.origin for c in cells]), np.concatenate([c.offsets for c in cells]),
                 np.concatenate([c.k for c in cells]), np.concatenate([c.traction for c in cells]))
    n = int(ref["steps"])
    bt.run(n // 2)
    bt.run(n - n // 2)
    bt.sync()
    for b in range(len(lats)):
        assert bt.box_steps(b) == n
        g = bt.read_populations(b).reshape(19, -1)
        o, off, _, _ = bt.read_vertices(b)
        disp = o[None, :].astype(np.float64) + off.astype(np.float64) - cells[b].positions64()[0]
        e_x = np.abs(disp - ref[f"b{b}_disp"]).max() / float(ref[f"b{b}_disp_max"])
        e_g = np.abs(g[:, ref[f"b{b}_sites"]] - ref[f"b{b}_pops"]).max() / float(ref[f"b{b}_pops_max"])
        print(f"batch box {b}: displacement {e_x:.2e}, populations {e_g:.2e}", flush=True)
        assert e_x <= TOL_LONG and e_g <= TOL_LONG, b
    bt.close()
