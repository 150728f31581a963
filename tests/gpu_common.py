"""Shared helpers of the device parity tests (device path vs FP64 oracle).

Both sides receive the same seeded inputs from `workloads`; the oracle sees
the float32 inputs promoted to float64.  Nothing here feeds a device output
back into the oracle except where a test compares integer work on the
device's own float32 positions (binning), which is the defined input of
that operation.
"""
import numpy as np

from oracle import lattice, step


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).max()
    return float(np.abs(a - b).max() / (s if s > 0 else 1.0))


def make_sim(w, cells=None, max_cells=None):
    from paper_2305_02752_amd import Simulation
    cells = cells if cells is not None else w.cells
    sim = Simulation(w.lattice, w.rest_pos, w.tri, max_cells=max_cells or max(cells.n, 1))
    if cells.n:
        sim.set_cells(cells.origin, cells.offsets, cells.k, cells.traction)
    return sim


def oracle_model(w, cells):
    return step.make_model(w.lattice, w.rest_pos.astype(np.float64), w.tri, cells.k.astype(np.float64),
                           None if cells.traction is None else cells.traction.astype(np.float64))


def oracle_state(g32, cells):
    return lattice.unshift(g32), cells.positions64()
