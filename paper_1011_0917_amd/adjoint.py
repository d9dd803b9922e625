"""Differentiable boosted-frame PIC loss as a ``torch.autograd.Function``.

The forward runs the taped simulation behind the C ABI (``bfpic_forward_loss``)
and the backward its reverse sweep (``pic_step_adjoint``): checkpoints every
``interval`` steps, recomputation of each segment, and the transposed step run
backwards.  The parameters are the laser amplitude a0 and the values of a
piecewise-linear lab density profile at fixed knots.  The loss is a wake-field
box mean, plus optionally the weighted mean lab energy of witness electrons
after the last step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import Simulation, make_laser


@dataclass
class PICLossSpec:
    """Everything of the run except the parameters a0 and the knot values."""
    cfg: object                     # Config
    capacity: int
    gamma_boost: float
    knots_z: list                   # lab positions of the density knots
    laser: dict                     # make_laser keywords except a0
    nsteps: int
    interval: int
    step_first: int
    step_last: int
    box: tuple                      # (i0, i1, j0, j1) Ez node box
    device: object = None
    witnesses: object = None        # (n, 6) float64 initial witness states (host or device)
    witness_weight: float = 0.0
    last: dict = field(default_factory=dict)


class BoostedPICLoss(torch.autograd.Function):
    """L(a0, n) = mean over the loss window of the box mean of Ez, plus
    witness_weight times the mean lab energy of the witnesses at the end."""

    @staticmethod
    def forward(ctx, a0, knots_n, spec: PICLossSpec):
        sim = Simulation(spec.cfg, capacity=spec.capacity, device=spec.device)
        laser = make_laser(**dict(spec.laser, a0=float(a0)))
        sim.init_boosted_plasma(spec.gamma_boost, knots_z=list(spec.knots_z),
                                knots_n=[float(v) for v in knots_n.detach().cpu()],
                                laser=laser)
        if spec.witnesses is not None:
            w = torch.as_tensor(spec.witnesses, dtype=torch.float64)
            sim.witness_bind(w.to(sim.device).clone().contiguous())
        loss = sim.forward_loss(spec.nsteps, spec.interval, spec.step_first, spec.step_last,
                                spec.box, witness_weight=spec.witness_weight)
        ctx.sim = sim
        ctx.nk = len(spec.knots_z)
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad):
        da0, dn = ctx.sim.adjoint(ctx.nk)
        ctx.sim.close()
        g = grad.detach().cpu().double()
        return (g * torch.tensor(da0, dtype=torch.float64),
                g * torch.tensor(dn, dtype=torch.float64), None)
