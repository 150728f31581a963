"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Everything here is input generation only: meshes, cell placement and
orientation, parameter draws and random lattice states.  None of the coupled
step's arithmetic lives here, so the oracle and the device path stay
independent while consuming identical inputs.
"""
from .mesh import icosphere, evans_fung, rbc_mesh, sphere_mesh  # noqa: F401
from .configs import (  # noqa: F401
    Lattice, Cells, Workload, K_REF, random_rotation, small_rotation,
    single_rbc_shear, dense_channel, large_suspension, batched_calibration,
    adjoint_boxes, tiny_periodic, random_shifted_populations, jitter_cells,
    place_cells, WORKLOADS,
)
