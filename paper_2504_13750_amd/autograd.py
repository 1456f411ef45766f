"""The probe loss of a trajectory as a differentiable torch function (one-step and
detailed models).

The paper makes its time integration differentiable by replacing automatic
differentiation of the step loop with the adjoint method behind a custom VJP (Sec. 6.1,
Eq. 6.1-6.5). Here the same role is played by janc_adjoint, which runs the trajectory
with checkpoints and sweeps it backwards in the HIP library: `probe_loss(W0, theta)`
returns L = sum_n dt sum_q w_q p(U^n at probe q) and, when torch asks for gradients,
dL/dW0 and, for the one-step model, dL/d(Q, E_a) from that same call (the adjoint runs
together with the forward pass, so backward is a scaling by the incoming gradient).
"""

import torch

from . import ONESTEP, DETAILED, make_physics, make_time


class _ProbeLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, W0, theta, jctx, grid, gamma, R, k, dt, nsteps, ckpt_every, probe_cell,
                probe_w):
        Q, Ea = (float(x) for x in theta.detach().cpu())
        phys = make_physics(gamma, R, Q, Ea, k)
        loss, gW, gth = jctx.adjoint(grid, phys, make_time(0.0, dt, 0.0), W0.detach().contiguous(),
                                     nsteps, ckpt_every, probe_cell, probe_w)
        fctx.save_for_backward(gW, gth.to(theta.device))
        return loss[0]

    @staticmethod
    def backward(fctx, g):
        gW, gth = fctx.saved_tensors
        return (g * gW, g * gth) + (None,) * 10


def probe_loss(ctx, grid, gamma, R, k, dt, W0, theta, nsteps, ckpt_every, probe_cell, probe_w):
    """Differentiable probe loss of nsteps fixed-dt steps.

    ctx: Context(ONESTEP) or Context(DETAILED, mech); grid: janc_grid (grid_of); W0
    (device, float64) [nfields, ny, nx] initial primitives of the model; theta (float64)
    [2] = (Q, E_a) of the one-step model (the detailed model has none: pass zeros, its
    gradient is zero); the other arguments as in Context.adjoint. Returns a 0-d tensor;
    gradients flow to W0 and theta."""
    if ctx.model not in (ONESTEP, DETAILED):
        raise ValueError("the adjoint covers the one-step and the detailed models")
    return _ProbeLoss.apply(W0, theta, ctx, grid, float(gamma), float(R), float(k), float(dt),
                            int(nsteps), int(ckpt_every), probe_cell, probe_w)
