"""torch.autograd wrapper of the adjoint form.

CoupledStepFn.apply(params, runner) returns the per-box losses of a batch of
independent single-cell boxes after n coupled steps; its backward returns
dL/dparams from the library's hand-written reverse sweep (checkpointed
recomputation), not from torch autograd.  params is a [B, 5] float64 tensor
of (k_link, k_bend, k_area, k_volume, tau) per box.
"""
from __future__ import annotations

import numpy as np
import torch

from .hemo import Simulation


class AdjointBoxes:
    """One Simulation per box with a fixed initial state that every forward
    evaluation restarts from.  Boxes of one shape run through the batched
    reverse-mode calls (every per-step kernel one launch over all boxes);
    otherwise each box runs on its own stream in turn."""

    def __init__(self, lattices, rest_pos, tri, cells, targets, n_steps, ckpt_every, device="cuda:0"):
        self.n_steps, self.ckpt_every = int(n_steps), int(ckpt_every)
        self.generation = 0   # forward evaluations so far; a backward belongs to the latest
        self.targets = np.asarray(targets, dtype=np.float64).reshape(len(lattices), 2)
        self.sims, self.streams, self.start = [], [], []
        for b, lat in enumerate(lattices):
            s = torch.cuda.Stream(device=device)
            with torch.cuda.stream(s):
                sim = Simulation(lat, rest_pos, tri, max_cells=1, device=device)
                c = cells[b]
                sim.set_cells(c.origin, c.offsets, c.k, c.traction)
                sim.init_equilibrium()
                sim.adj_bind(self.n_steps, self.ckpt_every)
                self.start.append(sim.checkpoint_save())
            self.sims.append(sim)
            self.streams.append(s)
        shape = {(lat.nx, lat.ny, lat.nz, tuple(lat.bc)) for lat in lattices}
        self.batched = len(shape) == 1

    def forward(self, params: np.ndarray) -> np.ndarray:
        self.generation += 1
        for b, sim in enumerate(self.sims):
            with torch.cuda.stream(self.streams[b]):
                sim.checkpoint_restore(self.start[b])
                sim.set_params(k=params[b, :4], tau=params[b, 4])
        if self.batched:
            return Simulation.adj_multi_forward(self.sims, self.targets)[:, 0]
        loss = np.empty(len(self.sims))
        for b, sim in enumerate(self.sims):
            with torch.cuda.stream(self.streams[b]):
                loss[b] = sim.adj_forward(self.targets[b])[0]
        return loss

    def backward(self) -> np.ndarray:
        if self.batched:
            return Simulation.adj_multi_backward(self.sims)[:, 0, :]
        g = np.empty((len(self.sims), 5))
        for b, sim in enumerate(self.sims):
            with torch.cuda.stream(self.streams[b]):
                g[b] = sim.adj_backward()[0]
        return g


class CoupledStepFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, runner: AdjointBoxes):
        loss = runner.forward(params.detach().cpu().numpy().astype(np.float64))
        ctx.runner = runner
        ctx.generation = runner.generation
        return torch.as_tensor(loss, dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, grad_loss: torch.Tensor):
        # the runner's contexts hold the checkpoints of its latest forward only
        if ctx.runner.generation != ctx.generation:
            raise RuntimeError("CoupledStepFn: the runner has evaluated another forward since this one; "
                               "its reverse sweep would belong to that forward (call backward first, or "
                               "use one runner per graph)")
        g = ctx.runner.backward()
        gl = grad_loss.detach().cpu().numpy()[:, None]
        return torch.as_tensor(gl * g, dtype=grad_loss.dtype, device=grad_loss.device), None
