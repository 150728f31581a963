"""Cell integration with separated time scales, float64 (oracle).

TEST INFRASTRUCTURE ONLY; see the package docstring.

Sec. 2.6: the cells are integrated by explicit Euler or by Adams-Bashforth,
and because the constitutive model is the costly part and the cell
equations tolerate larger steps than the fluid, the membrane forces are
evaluated less often than the fluid is advanced.  The paper gives neither
the Adams-Bashforth order nor how the separated steps are coupled; the
reading used here:
  * the membrane forces (with the pole traction) are recomputed at every
    `force_every`-th fluid step, counted from the start of the run, and the
    last ones are spread unchanged at the steps in between;
  * the vertices move at every fluid step with the velocity U^n
    interpolated in that step:
      Euler:  X^{n+1} = X^n + U^n
      AB2:    X^{n+1} = X^n + 3/2 U^n - 1/2 U^{n-1}
    (second-order Adams-Bashforth with unit step; its first step, which
    has no U^{n-1}, is an Euler step).
With force_every = 1 and Euler this is the plain coupled step.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import membrane, step


@dataclasses.dataclass
class CellState:
    """What the integration carries from one step to the next besides X."""
    Fv: np.ndarray | None = None       # membrane forces last evaluated
    U_prev: np.ndarray | None = None   # velocity of the previous step (AB2)
    steps: int = 0                     # fluid steps taken since the start


def advance(m: step.Model, f, X, st: CellState, force_every: int = 1, scheme: str = "euler"):
    """One fluid step with separated cell time scales; returns (f, X, st, info)."""
    if scheme not in ("euler", "ab2"):
        raise ValueError(scheme)
    if force_every < 1:
        raise ValueError(force_every)
    Fv = st.Fv
    if st.steps % force_every == 0 or Fv is None:
        Fv = (membrane.forces(X, m.k, m.topo, m.rest, m.traction) if X.shape[0]
              else np.zeros_like(X))
    f_new, U, info = step.fluid_step(m, f, X, Fv, st.steps)
    if scheme == "ab2" and st.U_prev is not None:
        X_new = X + 1.5 * U - 0.5 * st.U_prev
    else:
        X_new = X + U
    return f_new, X_new, CellState(Fv=Fv, U_prev=U, steps=st.steps + 1), info


def run(m: step.Model, f, X, n: int, force_every: int = 1, scheme: str = "euler",
        st: CellState | None = None):
    """n steps from (f, X); returns (f, X, state)."""
    st = CellState() if st is None else st
    for _ in range(n):
        f, X, st, _ = advance(m, f, X, st, force_every, scheme)
    return f, X, st
