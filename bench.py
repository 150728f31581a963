#!/usr/bin/env python3
"""Throughput of the coupled D3Q19 + IBM + membrane step on one MI355X.

Workload (default): the large-suspension run -- 256 x 256 x 512 fully
periodic lattice (33.5M sites), 18,600 biconcave RBCs of 642 vertices
(11.9M vertices, haematocrit ~44%), body force along z, tau = 1, cells
binned to 8^3 tiles each step.  Inputs are synthetic (seeded force-bias
packing, uniform random orientations); populations start at rest.

A step is one pass of the whole coupled update through libhemo: the per-cell
kernel (vertex move of the previous step, membrane forces, binning) and the
per-tile lattice pass (IBM spread, collide + stream, IBM interpolation); the
move that closes the last step runs once at the end.  The force and velocity
fields stay on chip (field output off).
The timed region runs exactly --steps steps with inputs resident in HBM,
bracketed by device synchronisation; per-kernel device time inside the same
region comes from events recorded on the library's stream.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0          # MI355X HBM3E peak
BYTES_PER_SITE = 152            # 19 float32 populations read + written
BYTES_PER_VERTEX = 24           # float32 position read + written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lattice_pass_traffic.json")
LATTICE_SOURCES = ("ibm.hip", "ibm_dev.h", "lbm_dev.h", "common.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in LATTICE_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2305_02752_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(n_sites: int):
    """HBM bytes per launch of the lattice pass from committed rocprofv3 PMC
    counters, valid only for the kernel source they were taken on."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if rec.get("source_hash") != kernel_source_hash() or rec.get("n_sites") != n_sites:
        return None
    return float(rec["bytes_per_launch"])


def cpu_baseline(w, steps: int = 3, side: int = 64):
    """Time the FP64 oracle on a bounded sample of the same suspension: a
    side^3 periodic sub-box holding the cells whose centres fall inside it."""
    from threadpoolctl import threadpool_limits

    from oracle import lattice, step
    from workloads.configs import Cells, Lattice

    lat = w.lattice
    cen = w.cells.positions64().mean(axis=1)
    sel = np.all((cen >= 0) & (cen < side), axis=1)
    cells = Cells(origin=w.cells.origin[sel], offsets=w.cells.offsets[sel], k=w.cells.k[sel])
    sub = Lattice(side, side, side, tau=lat.tau, body_force=lat.body_force)
    m = step.make_model(sub, w.rest_pos.astype(np.float64), w.tri, cells.k.astype(np.float64))
    f = lattice.init_equilibrium(sub.shape)
    X = cells.positions64()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(steps):
            f, X, _ = step.step(m, f, X)
        dt = time.perf_counter() - t0
    nv = X.shape[0] * X.shape[1]
    return {
        "value": sub.n_sites * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} steps of a {side}^3 periodic sub-box with the {int(sel.sum())} cells "
                  f"({nv} vertices) centred in it, float64 NumPy, 1 thread",
        "vertex_updates_per_s": nv * steps / dt,
        "s_per_step": dt / steps,
    }


def copy_bandwidth(torch, nbytes: int = 4 << 30, reps: int = 5):
    """GB/s (read + write bytes) of the library's streaming copy kernel and,
    beside it, of torch's device-to-device copy (a hipMemcpyAsync)."""
    from paper_2305_02752_amd.hemo import device_copy
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    lib = timed(lambda: device_copy(b.data_ptr(), a.data_ptr(), nbytes, s))
    memcpy = timed(lambda: b.copy_(a))
    del a, b
    torch.cuda.empty_cache()
    return lib, memcpy


def bench_separated(sim, n_sites: int, warmup: int, steps: int, force_every: int = 10):
    """The same suspension with separated cell time scales: membrane forces
    every `force_every` steps (held in between), Adams-Bashforth moves."""
    sim.set_integration(force_every, "ab2")
    sim.step(warmup)
    sim.sync()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    dt = time.perf_counter() - t0
    prof = sim.profile_read()
    sim.profile(False)
    sim.set_integration(1, "euler")
    return {"force_every": force_every, "scheme": "ab2", "steps": steps,
            "ms_per_step": dt / steps * 1e3, "MLUPS": n_sites * steps / dt / 1e6,
            "kernel_ms": {k: ms / max(n, 1) for k, (ms, n) in prof.items()}}


def bench_fluid_only(torch, w, warmup: int, steps: int):
    """The same lattice with no cells: the fused lattice pass reduced to
    pull-stream + collide, against the same 152 B/site and the same peak.
    Splits the coupled pass's time into its streaming part and its IBM
    phases."""
    from paper_2305_02752_amd import Simulation
    lat = w.lattice
    sim = Simulation(lat, w.rest_pos, w.tri, max_cells=1)
    sim.init_equilibrium()
    sim.set_field_output(False)
    sim.step(warmup)
    sim.sync()
    sim.profile(True)
    sim.step(steps)
    sim.sync()
    ms, n = sim.profile_read()["lattice"]
    sim.close()
    avg = ms / max(n, 1)
    gbps = BYTES_PER_SITE * lat.n_sites / (avg * 1e-3) / 1e9
    return {"steps": steps, "lattice_pass_ms": avg, "achieved_GBps": gbps, "frac": gbps / PEAK_HBM_GBPS}


def bench_interior(sim, n_sites: int, warmup: int, steps: int, ratio: float = 5.0):
    """The same suspension with the cytosol `ratio` times as viscous as the
    plasma: the sites inside the cells are marked every step and relax with
    the interior relaxation time."""
    sim.set_interior_viscosity(ratio)
    sim.step(warmup)
    sim.sync()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    dt = time.perf_counter() - t0
    prof = sim.profile_read()
    sim.profile(False)
    sim.set_interior_viscosity(1.0)
    return {"ratio": ratio, "steps": steps, "ms_per_step": dt / steps * 1e3,
            "MLUPS": n_sites * steps / dt / 1e6,
            "kernel_ms": {k: ms / max(n, 1) for k, (ms, n) in prof.items()}}


def bench_mixture(sim, w, n_sites: int, warmup: int, steps: int, stiff_fraction: float = 0.5,
                  link_scale: float = 5.0, ratio_healthy: float = 5.0, ratio_stiff: float = 10.0):
    """Stiffened/healthy mixture of the same suspension (Sec. 3.4: stiffened
    cells scale the link coefficient and the internal viscosity ratio; the
    paper gives no factors, these are readings): every other cell stiffened,
    one interior viscosity ratio per cell."""
    n = w.cells.n
    stiff = (np.arange(n) % int(round(1.0 / stiff_fraction))) == 0
    k = w.cells.k.astype(np.float32).copy()
    k[stiff, 0] *= link_scale
    sim.set_params(k=k)
    sim.set_cell_viscosity(np.where(stiff, ratio_stiff, ratio_healthy))
    sim.step(warmup)
    sim.sync()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    dt = time.perf_counter() - t0
    prof = sim.profile_read()
    sim.profile(False)
    sim.set_interior_viscosity(1.0)
    sim.set_params(k=w.cells.k)
    return {"stiff_fraction": float(stiff.mean()), "link_scale": link_scale,
            "ratios": [ratio_healthy, ratio_stiff], "steps": steps, "ms_per_step": dt / steps * 1e3,
            "MLUPS": n_sites * steps / dt / 1e6,
            "kernel_ms": {kk: ms / max(c, 1) for kk, (ms, c) in prof.items()}}


def bench_lees_edwards(torch, w, warmup: int, steps: int, u_le: float = 0.02):
    """The large suspension as a boundary-free shear: the same lattice and
    cells with Lees-Edwards images (gradient z, flow x, image velocity u_le)
    instead of the body force; then the same with an interior viscosity
    ratio of 5."""
    import dataclasses

    from paper_2305_02752_amd import Simulation
    lat = dataclasses.replace(w.lattice, body_force=(0.0, 0.0, 0.0), lees_edwards_u=u_le)
    sim = Simulation(lat, w.rest_pos, w.tri, max_cells=w.cells.n)
    sim.set_cells(w.cells.origin, w.cells.offsets, w.cells.k, None)
    sim.init_equilibrium()
    sim.set_field_output(False)
    n = lat.nx * lat.ny * lat.nz

    def timed():
        sim.step(warmup)
        sim.sync()
        sim.profile(True)
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        dt = time.perf_counter() - t0
        prof = sim.profile_read()
        sim.profile(False)
        return {"ms_per_step": dt / steps * 1e3, "MLUPS": n * steps / dt / 1e6,
                "kernel_ms": {k: ms / max(c, 1) for k, (ms, c) in prof.items()}}

    out = {"u_le": u_le, "steps": steps, **timed()}
    # the same shear with the cytosol five times as viscous as the plasma
    sim.set_interior_viscosity(5.0)
    out["interior_ratio_5"] = timed()
    sim.close()
    return out


def bench_packing(torch, n: int = 1_000_000, iters: int = 20):
    """Force-bias packing of a million random surrogate ellipsoids (RBC
    enclosing ellipsoids filling 35% of a periodic cube): time per
    iteration and the overlap before and after."""
    from paper_2305_02752_amd import Packer
    from workloads.configs import RBC_SURROGATE, ellipsoid_suspension

    c, R, s, side = ellipsoid_suspension(n=n)
    pk = Packer((side,) * 3, (True,) * 3, max_semi=max(RBC_SURROGATE), eta=0.03, max_move=1.0, quad=8)
    dev = torch.device("cuda:0")
    tc = torch.tensor(c, device=dev)
    tr = torch.tensor(R.reshape(-1, 9), device=dev)
    ts = torch.tensor(s, device=dev)
    before = pk.run_device(tc, tr, ts, 0)
    pk.run_device(tc, tr, ts, 2, measure=False)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk.run_device(tc, tr, ts, iters, measure=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    after = pk.run_device(tc, tr, ts, 0)
    return {"ellipsoids": n, "side": side, "volume_fraction": 0.35, "quad": 8, "iterations": iters,
            "ms_per_iteration": dt / iters * 1e3, "ellipsoid_updates_per_s": n * iters / dt,
            "overlap_volume_before": before[0], "overlapping_pairs_before": int(before[1]),
            "overlap_volume_after": after[0], "overlapping_pairs_after": int(after[1]),
            "iterations_before_after": 2 + iters}


def bench_small(torch):
    """The single-cell shear box (32^3, 500 steps) and the dense channel
    (128x64x64, 220 cells, 1000 steps): whole runs, timed per step."""
    from paper_2305_02752_amd import Simulation
    from workloads import dense_channel, single_rbc_shear

    out = {}
    for w in (single_rbc_shear(), dense_channel()):
        sim = Simulation(w.lattice, w.rest_pos, w.tri, max_cells=w.cells.n)
        sim.set_cells(w.cells.origin, w.cells.offsets, w.cells.k, w.cells.traction)
        sim.init_equilibrium()
        sim.set_field_output(False)
        sim.step(20)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(w.steps)
        sim.sync()
        dt = time.perf_counter() - t0
        n = w.lattice.nx * w.lattice.ny * w.lattice.nz
        nv = w.cells.n * w.rest_pos.shape[0]
        out[w.name] = {"steps": w.steps, "us_per_step": dt / w.steps * 1e6,
                       "MLUPS": n * w.steps / dt / 1e6, "vertex_updates_per_s": nv * w.steps / dt,
                       "launches_per_step": 2}
        sim.close()
    return out


def bench_batched(torch, seed: int = 3, steps: int = 2000, warmup: int = 20):
    """Batched calibration workload: 256 single-cell boxes (sides U{24..48})
    advanced together, one persistent launch per run, tiling autotuned."""
    import tempfile

    from paper_2305_02752_amd import Batch
    from workloads import batched_calibration

    w = batched_calibration(seed=seed)
    cells = w.cells
    bt = Batch(w.lattice, w.rest_pos, w.tri)
    bt.set_cells(np.concatenate([c.origin for c in cells]), np.concatenate([c.offsets for c in cells]),
                 np.concatenate([c.k for c in cells]), np.concatenate([c.traction for c in cells]))
    with tempfile.TemporaryDirectory() as d:
        choice = bt.autotune(os.path.join(d, "tiling.txt"), trial_steps=10)
    bt.run(warmup)
    bt.sync()
    n0 = bt.launches()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.run(steps)
    bt.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sites = sum(l.n_sites for l in w.lattice)
    nv = len(cells) * w.rest_pos.shape[0]
    return {"workload": w.name, "boxes": len(cells), "sites": sites, "vertices": nv, "steps": steps,
            "launches": bt.launches() - n0, "ms_per_step": dt / steps * 1e3,
            "MLUPS": sites * steps / dt / 1e6, "vertex_updates_per_s": nv * steps / dt,
            "hbm_frac": (BYTES_PER_SITE * sites + BYTES_PER_VERTEX * nv) * steps / dt / 1e9 / PEAK_HBM_GBPS,
            "tiling": {**choice, **bt.tiling()}}


def bench_adjoint(torch, boxes: int = 64, seed: int = 4):
    """Adjoint workload (48^3 sheared boxes with pole traction, 2000 steps,
    checkpoint every 100): gradients of the cell-shape loss with respect to
    (k_link, k_bend, k_area, k_volume, tau) of `boxes` of the 64 boxes (all
    of them by default), timed through the torch form itself:
    CoupledStepFn.apply(params, runner) and .backward(), whose runner drives
    the batched reverse-mode calls (one launch per kernel over all boxes).
    The cost of a gradient is reported against the batched persistent form
    advancing the same boxes by the same number of steps."""
    import tempfile

    from paper_2305_02752_amd import Batch
    from paper_2305_02752_amd.autograd import AdjointBoxes, CoupledStepFn
    from workloads import adjoint_boxes

    w = adjoint_boxes(seed=seed)
    n, ck = w.steps, w.extra["ckpt_every"]
    lats, cells = w.lattice[:boxes], w.cells[:boxes]
    # the forward it is measured against: the batched persistent form
    bt = Batch(lats, w.rest_pos, w.tri)
    bt.set_cells(np.concatenate([c.origin for c in cells]), np.concatenate([c.offsets for c in cells]),
                 np.concatenate([c.k for c in cells]), np.concatenate([c.traction for c in cells]))
    with tempfile.TemporaryDirectory() as d:
        bt.autotune(os.path.join(d, "tiling.txt"), trial_steps=10)
    bt.run(20)
    bt.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.run(n)
    bt.sync()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    bt.close()

    runner = AdjointBoxes(lats, w.rest_pos, w.tri, cells, w.extra["targets"][:boxes], n, ck)
    p0 = np.array([np.concatenate([c.k[0], [lat.tau]]) for c, lat in zip(cells, lats)])
    params = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = CoupledStepFn.apply(params, runner)
    torch.cuda.synchronize()
    t_af = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss.sum().backward()
    torch.cuda.synchronize()
    t_bw = time.perf_counter() - t0
    g = params.grad.numpy()
    for sim in runner.sims:
        sim.close()
    return {"workload": w.name, "boxes_timed": boxes, "boxes_in_workload": len(w.cells), "steps": n,
            "ckpt_every": ck, "batched_calls": bool(runner.batched), "grads_per_s": boxes / (t_af + t_bw),
            "t_forward_batched_form_s": t_fwd, "t_adjoint_forward_s": t_af, "t_backward_s": t_bw,
            "t_grad_over_t_forward": (t_af + t_bw) / t_fwd,
            "finite": bool(np.all(np.isfinite(g)) and np.all(np.isfinite(loss.detach().numpy())))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and adjoint forms")
    ap.add_argument("--adjoint-boxes", type=int, default=64)
    ap.add_argument("--packing-only", action="store_true",
                    help="time only the force-bias packing of a million ellipsoids (one JSON line)")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched calibration form (one JSON line)")
    ap.add_argument("--fluid-only", action="store_true",
                    help="time only the lattice pass of the large suspension's lattice without cells "
                         "(one JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.packing_only:
        print(json.dumps({"force_bias_packing": bench_packing(torch)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_calibration": bench_batched(torch)}), flush=True)
        return
    if args.fluid_only:
        from workloads import rbc_mesh
        from workloads.configs import Lattice, Workload
        rest, tri = rbc_mesh(3, 16.0)   # the suspension's cell mesh (unused: no cells)
        lat = Lattice(256, 256, 512, tau=1.0, body_force=(0.0, 0.0, 1e-6))
        w = Workload("large_suspension_256x256x512_without_cells", lat, rest.astype(np.float32), tri,
                     None, args.steps)
        print(json.dumps({"fluid_only_lattice_pass": bench_fluid_only(torch, w, args.warmup, args.steps)}),
              flush=True)
        return

    from paper_2305_02752_amd import Simulation
    from workloads import large_suspension

    t = time.time()
    w = large_suspension(seed=args.seed)
    lat = w.lattice
    n_sites = lat.n_sites
    n_vert = w.cells.n * w.rest_pos.shape[0]
    log(f"workload {w.name}: {n_sites} sites, {w.cells.n} cells, {n_vert} vertices, "
        f"packing residual {w.extra['pack_residual']:.2f} lu, built in {time.time() - t:.1f}s")

    copy_gbps, memcpy_gbps = copy_bandwidth(torch)
    log(f"library copy kernel: {copy_gbps:.0f} GB/s; hipMemcpyAsync device to device: {memcpy_gbps:.0f} GB/s")

    sim = Simulation(lat, w.rest_pos, w.tri, max_cells=w.cells.n)
    sim.set_cells(w.cells.origin, w.cells.offsets, w.cells.k, None)
    sim.init_equilibrium()
    sim.set_field_output(False)
    log(f"workspace {sim.workspace_bytes / 2**30:.2f} GiB")

    sim.step(args.warmup)
    sim.sync()
    log(f"warmup {args.warmup} steps done")

    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    sim.profile(False)
    sim.sync()
    dt = t1 - t0
    log(f"timed {args.steps} steps in {dt:.3f}s")
    for k, (ms, n) in prof.items():
        log(f"  {k:15s} {ms / max(n, 1):8.3f} ms/launch  ({n} launches)")

    ms_step = dt / args.steps * 1e3
    mlups = n_sites * args.steps / dt / 1e6
    vups = n_vert * args.steps / dt
    b_step = BYTES_PER_SITE * n_sites + BYTES_PER_VERTEX * n_vert
    step_frac = b_step * args.steps / dt / 1e9 / PEAK_HBM_GBPS

    ms_cs, n_cs = prof["lattice"]
    avg_s = ms_cs / n_cs * 1e-3
    alg_bytes = BYTES_PER_SITE * n_sites
    achieved = alg_bytes / avg_s / 1e9
    traffic = measured_traffic(n_sites)
    roofline = {"bound": "hbm", "kernel": "lattice_pass", "achieved": achieved,
                "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS,
                "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
                "avg_launch_ms": avg_s * 1e3}

    tss = interior = mixture = None
    if not args.no_extra:
        tss = bench_separated(sim, n_sites, args.warmup, args.steps)
        log(f"separated time scales (forces every {tss['force_every']}, {tss['scheme']}): "
            f"{tss['ms_per_step']:.3f} ms/step, {tss['MLUPS']:.0f} MLUPS")
        interior = bench_interior(sim, n_sites, args.warmup, args.steps)
        log(f"interior viscosity ratio {interior['ratio']}: {interior['ms_per_step']:.3f} ms/step, "
            f"marking {interior['kernel_ms']['interior']:.3f} ms")
        mixture = bench_mixture(sim, w, n_sites, args.warmup, args.steps)
        log(f"stiffened/healthy mixture: {mixture['ms_per_step']:.3f} ms/step, "
            f"marking {mixture['kernel_ms']['interior']:.3f} ms")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    batched = adj = None
    if not args.no_extra:
        log("batched calibration form ...")
        batched = bench_batched(torch)
        log(f"batched: {batched['ms_per_step']:.3f} ms/step, {batched['MLUPS']:.0f} MLUPS, "
            f"{batched['launches']} launch(es), tiling {batched['tiling']}")
        torch.cuda.empty_cache()
        log("adjoint form ...")
        adj = bench_adjoint(torch, boxes=args.adjoint_boxes)
        torch.cuda.empty_cache()
        log(f"adjoint: {adj['grads_per_s']:.2f} gradients/s over {adj['boxes_timed']} boxes, "
            f"t_grad/t_fwd {adj['t_grad_over_t_forward']:.2f}")

    small = lees = packing = fluid = None
    if not args.no_extra:
        log("the same lattice without cells ...")
        fluid = bench_fluid_only(torch, w, args.warmup, args.steps)
        torch.cuda.empty_cache()
        log(f"  lattice pass {fluid['lattice_pass_ms']:.3f} ms, {fluid['achieved_GBps']:.0f} GB/s "
            f"({100 * fluid['frac']:.1f}% of peak)")
        log("force-bias packing of a million ellipsoids ...")
        packing = bench_packing(torch)
        torch.cuda.empty_cache()
        log(f"  {packing['ms_per_iteration']:.3f} ms/iteration, overlapping pairs "
            f"{packing['overlapping_pairs_before']} -> {packing['overlapping_pairs_after']}")
        log("Lees-Edwards shear of the same suspension ...")
        lees = bench_lees_edwards(torch, w, args.warmup, args.steps)
        torch.cuda.empty_cache()
        log(f"  {lees['ms_per_step']:.3f} ms/step, {lees['MLUPS']:.0f} MLUPS; with interior viscosity "
            f"{lees['interior_ratio_5']['ms_per_step']:.3f} ms/step")
        log("single-cell shear and dense channel ...")
        small = bench_small(torch)
        for k, v in small.items():
            log(f"  {k}: {v['us_per_step']:.1f} us/step, {v['MLUPS']:.0f} MLUPS")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        cpu = cpu_baseline(w, steps=args.cpu_steps)
        log(f"oracle: {cpu['value']:.3f} MLUPS ({cpu['s_per_step']:.2f} s/step)")

    out = {
        "metric": "coupled-step MLUPS",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": [lat.nx, lat.ny, lat.nz], "cells": w.cells.n,
                   "vertices": n_vert, "tau": lat.tau, "ibm_kernel": "phi4", "tile": 8},
        "vertex_updates_per_s": vups,
        "step_hbm_frac": step_frac,
        "step_algorithmic_bytes": b_step,
        "copy_kernel_GBps": copy_gbps,
        "memcpy_GBps": memcpy_gbps,
        "kernel_ms": {k: ms / max(n, 1) for k, (ms, n) in prof.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "separated_time_scales": tss,
        "interior_viscosity": interior,
        "stiffened_mixture": mixture,
        "small_workloads": small,
        "lees_edwards_shear": lees,
        "force_bias_packing": packing,
        "fluid_only_lattice_pass": fluid,
        "batched_calibration": batched,
        "adjoint": adj,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
