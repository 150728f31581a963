#!/usr/bin/env python3
"""Write the stored reference values of the long-horizon parity tests.

Calls only the FP64 oracle (`oracle/`) and the seeded input generators
(`workloads/`); nothing here touches the device library.

  dense_channel  the dense channel suspension (128 x 64 x 64, walls at the
                 y bounds, body force along x, 220 cells) after 1000 steps
                 from rest: displacement of every 8th vertex of every cell,
                 shifted populations at 4096 seeded sites, and the maxima of
                 the full fields (the denominators of the relative errors).
  adjoint        central finite-difference gradients of the cell-shape loss
                 for two boxes of the adjoint workload (48^3, sheared, pole
                 traction, 2000 steps), step h = 1e-4 |p_j|, with the loss at
                 p and whether the extreme vertices of both diameters are
                 the same at p +- h (so that the difference quotient is taken
                 on one smooth branch of the max/min).
  adjoint_cs     the same gradients by the complex step (the oracle's
                 difference-free gradient), one run per parameter.
  batch_1000     the five small batched-form boxes after 1000 steps from
                 rest: per box the displacement of every vertex, shifted
                 populations at 2048 seeded sites and the full-field maxima.

Usage: python tests/golden/make_goldens.py {dense_channel|adjoint|adjoint_cs|batch_1000} [--jobs N]
"""
from __future__ import annotations

import argparse
import dataclasses
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import adjoint as oadj  # noqa: E402
from oracle import lattice, step  # noqa: E402
from workloads import adjoint_boxes, dense_channel  # noqa: E402

DENSE_FILE = os.path.join(HERE, "dense_channel_1000.npz")
ADJ_FILE = os.path.join(HERE, "adjoint_full_boxes_fd.npz")
ADJ_CS_FILE = os.path.join(HERE, "adjoint_full_boxes_cs.npz")
BATCH_FILE = os.path.join(HERE, "batch_boxes_1000.npz")
BATCH_SEED, BATCH_STEPS = 2, 1000
ADJ_BOXES = (0, 1)
FD_EPS = 1e-4


def make_dense_channel():
    w = dense_channel()
    m = step.make_model(w.lattice, w.rest_pos.astype(np.float64), w.tri, w.cells.k.astype(np.float64), None)
    f = lattice.init_equilibrium(w.lattice.shape)
    X0 = w.cells.positions64()
    X = X0
    t0 = time.time()
    for i in range(w.steps):
        f, X, _ = step.step(m, f, X, i)
        if (i + 1) % 50 == 0:
            print(f"dense channel: step {i + 1}/{w.steps}, {time.time() - t0:.0f}s", flush=True)
    disp = X - X0
    g = lattice.shifted(f)
    rng = np.random.default_rng(12345)
    n = w.lattice.n_sites
    sites = np.sort(rng.choice(n, 4096, replace=False))
    np.savez_compressed(
        DENSE_FILE,
        steps=w.steps,
        vertex_stride=8,
        displacement=disp[:, ::8, :],
        displacement_max=np.abs(disp).max(),
        sites=sites,
        populations=g.reshape(19, -1)[:, sites],
        populations_max=np.abs(g).max(),
    )
    print("wrote", DENSE_FILE, flush=True)


def _extremes(X):
    return np.array([np.argmax(X[:, 0]), np.argmin(X[:, 0]), np.argmax(X[:, 1]), np.argmin(X[:, 1])])


def _adj_job(args):
    b, j, sgn = args
    w = adjoint_boxes()
    c = w.cells[b]
    k = c.k[0].astype(np.float64)
    p = np.concatenate([k, [w.lattice[b].tau]])
    h = FD_EPS * abs(p[j]) if j >= 0 else 0.0
    q = p.copy()
    if j >= 0:
        q[j] += sgn * h
    L, X = oadj.run_loss(w.lattice[b], w.rest_pos, w.tri, c.positions64()[0], q[:4],
                         c.traction[0].astype(np.float64), q[4], w.steps, w.extra["targets"][b])
    print(f"adjoint box {b} param {j} sign {sgn:+.0f}: loss {L:.10e}", flush=True)
    return (b, j, sgn), (L, _extremes(X), h)


def make_adjoint(jobs: int):
    from multiprocessing import Pool

    work = [(b, -1, 0.0) for b in ADJ_BOXES] + [(b, j, s) for b in ADJ_BOXES for j in range(5) for s in (1.0, -1.0)]
    with Pool(jobs) as pool:
        res = dict(pool.map(_adj_job, work, chunksize=1))
    w = adjoint_boxes()
    out = {"boxes": np.array(ADJ_BOXES), "eps": FD_EPS, "steps": w.steps, "ckpt_every": w.extra["ckpt_every"]}
    loss, grad, same, params = [], [], [], []
    for b in ADJ_BOXES:
        L0, e0, _ = res[(b, -1, 0.0)]
        g = np.zeros(5)
        ok = np.zeros(5, dtype=bool)
        for j in range(5):
            Lp, ep, h = res[(b, j, 1.0)]
            Lm, em, _ = res[(b, j, -1.0)]
            g[j] = (Lp - Lm) / (2 * h)
            ok[j] = np.array_equal(ep, e0) and np.array_equal(em, e0)
        c = w.cells[b]
        params.append(np.concatenate([c.k[0].astype(np.float64), [w.lattice[b].tau]]))
        loss.append(L0)
        grad.append(g)
        same.append(ok)
    out.update(loss=np.array(loss), fd_grad=np.array(grad), extremes_same=np.array(same), params=np.array(params))
    np.savez(ADJ_FILE, **out)
    print("wrote", ADJ_FILE, out, flush=True)


def _cs_job(args):
    b, j = args
    w = adjoint_boxes()
    c = w.cells[b]
    p = np.concatenate([c.k[0].astype(np.float64), [w.lattice[b].tau]])
    h = 1e-30 * abs(p[j])
    q = p.astype(np.complex128)
    q[j] += 1j * h
    L, _ = oadj.run_loss(w.lattice[b], w.rest_pos, w.tri, c.positions64()[0], q[:4],
                         c.traction[0].astype(np.float64), q[4], w.steps, w.extra["targets"][b])
    print(f"adjoint box {b} complex step param {j}: dL/dp {L.imag / h:.10e}", flush=True)
    return (b, j), L.imag / h


def make_adjoint_cs(jobs: int):
    from multiprocessing import Pool

    work = [(b, j) for b in ADJ_BOXES for j in range(5)]
    with Pool(jobs) as pool:
        res = dict(pool.map(_cs_job, work, chunksize=1))
    grad = np.array([[res[(b, j)] for j in range(5)] for b in ADJ_BOXES])
    np.savez(ADJ_CS_FILE, boxes=np.array(ADJ_BOXES), steps=adjoint_boxes().steps, cs_grad=grad)
    print("wrote", ADJ_CS_FILE, grad, flush=True)


def _batch_job(b):
    from workloads.configs import small_batch_boxes
    lats, rest, tri, cells = small_batch_boxes(BATCH_SEED)
    l, c = lats[b], cells[b]
    m = step.make_model(l, rest.astype(np.float64), tri, c.k.astype(np.float64), c.traction.astype(np.float64))
    X0 = c.positions64()
    f, X = step.run(m, lattice.init_equilibrium(l.shape), X0, BATCH_STEPS)
    g = lattice.shifted(f).reshape(19, -1)
    sites = np.sort(np.random.default_rng(100 + b).choice(l.n_sites, 2048, replace=False))
    disp = (X - X0)[0]
    print(f"batch box {b}: done", flush=True)
    return b, dict(disp=disp, disp_max=np.abs(disp).max(), sites=sites, pops=g[:, sites],
                   pops_max=np.abs(g).max())


def make_batch(jobs: int):
    from multiprocessing import Pool
    with Pool(jobs) as pool:
        res = dict(pool.map(_batch_job, range(5), chunksize=1))
    out = {"seed": BATCH_SEED, "steps": BATCH_STEPS}
    for b in range(5):
        for k, v in res[b].items():
            out[f"b{b}_{k}"] = v
    np.savez_compressed(BATCH_FILE, **out)
    print("wrote", BATCH_FILE, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["dense_channel", "adjoint", "adjoint_cs", "batch_1000"])
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    if a.what == "dense_channel":
        make_dense_channel()
    elif a.what == "adjoint":
        make_adjoint(a.jobs)
    elif a.what == "adjoint_cs":
        make_adjoint_cs(a.jobs)
    else:
        make_batch(a.jobs)


if __name__ == "__main__":
    main()
