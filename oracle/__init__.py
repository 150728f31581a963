"""Plain FP64 CPU oracle for the coupled fluid-cell time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check and the benchmark's CPU
baseline use it.  It shares no code, tables or constants with the device
library; both consume the seeded inputs of `workloads`.

The oracle follows the paper's model statement:
  * lattice Boltzmann BGK on D3Q19 (Sec. 2.2: update equation, density and
    velocity moments, second-order equilibrium, c_s^2 = 1/3,
    nu = c_s^2 (tau - 1/2));
  * immersed-boundary coupling through external force terms with
    interpolation in both directions (Sec. 2.3);
  * membrane force F_total = F_link + F_bend + F_area + F_volume (Sec. 2.3);
  * explicit Euler integration of the vertices (Sec. 2.6);
  * the force-bias packing of surrogate ellipsoids (Sec. 2.4).
Where the paper leaves a choice open the oracle uses the readings listed in
each module's docstring.

Parity pinned for: lattice (Couette, Poiseuille, conservation, equilibrium
moments), IBM (kernel moments, transpose identity), membrane (rest, rigid
motions, energy gradient, convex-hull volume), binning (brute force), coupled
step (uniform translation), interior marking (sphere inside/outside, ray
direction independence), packing (lens volume, containment, balanced
pushes).  Parity unpinned: agreement of the membrane force
forms with the paper's own implementation, whose formulas are in a reference
that is not reproduced in the paper.
"""
from . import lattice, ibm, membrane, binning, step, adjoint  # noqa: F401
