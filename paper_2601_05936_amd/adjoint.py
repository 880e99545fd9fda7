"""Differentiation of the gas centroid after n steps with respect to the
surface tension and the initial level set (reverse mode through the C ABI,
with time checkpoints).

`RiseHeight.apply(sigma, phi0, params, steps, every, axis)` returns the
centroid coordinate `axis` of the gas after `steps` steps as a 0-d float64
tensor; its backward pass reverses the run segment by segment: reload the
checkpoint, re-run the segment with the (deterministic) forward kernels
while recording it, reverse it.  Only the arithmetic of the reverse kernels
runs outside the forward path; everything is on the GPU.
"""
from __future__ import annotations

import torch

from .lsb import Sim


def _run_forward(params: dict, sigma: float, phi0: torch.Tensor, steps: int, every: int, rho0=None, u0=None):
    p = dict(params, sigma=float(sigma))
    sim = Sim(p).init(phi0, rho0, u0)
    ckpts = []
    for s0 in range(0, steps, every):
        ckpts.append(sim.save_state())
        sim.step(min(every, steps - s0))
    return sim, ckpts


def reverse_centroid(sim: Sim, ckpts, steps: int, every: int, axis: int, phi0, u0=None, rho0_given=False):
    """dL/dphi0 (device tensor) and dL/dsigma for L = centroid[axis] after
    `steps` steps, from the checkpoints of the forward run."""
    sim.adjoint_bind(every)
    nseg = len(ckpts)
    for s in reversed(range(nseg)):
        n = min(every, steps - s * every)
        sim.load_state(ckpts[s])
        sim.adjoint_record(n)
        if s == nseg - 1:
            sim.adjoint_seed_centroid(axis)
        sim.adjoint_reverse()
    return sim.adjoint_initial(phi0, u0, rho0_given)


class RiseHeight(torch.autograd.Function):
    """Gas centroid coordinate after `steps` steps as a function of sigma
    (0-d tensor) and phi0 (device tensor of N values)."""

    @staticmethod
    def forward(ctx, sigma, phi0, params, steps, every, axis):
        sim, ckpts = _run_forward(params, float(sigma), phi0, steps, every)
        L = float(sim.integrals()["centroid"][axis])
        ctx.state = (sim, ckpts, phi0.detach(), steps, every, axis)
        return torch.tensor(L, dtype=torch.float64, device=phi0.device)

    @staticmethod
    def backward(ctx, gL):
        sim, ckpts, phi0, steps, every, axis = ctx.state
        dphi0, dsig = reverse_centroid(sim, ckpts, steps, every, axis, phi0)
        g = gL.to(torch.float64)
        dsigma = (g * dsig).reshape(())
        return dsigma, (g * dphi0).reshape(phi0.shape), None, None, None, None
