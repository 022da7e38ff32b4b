"""Differentiable leapfrog rollouts through libbhx.

``rollout(x0, v0, m, ctx, dt, nsteps, ...)`` returns the positions and
velocities after ``nsteps`` kick-drift-kick steps (with a0 = A(x0)) as a
``torch.autograd.Function``: the backward pass gives gradients with respect to
x0, v0 and the masses. The forward keeps a checkpoint (x, v, a) every
``checkpoint_every`` steps; the backward recomputes each segment's positions
and runs the adjoint steps in the library (bh_leapfrog_vjp), then one force
VJP at x0 (bh_accel_vjp) for the dependence of a0 on x0. With
``keep_positions`` the forward keeps the positions after every step instead
(24 bytes per body and step of device memory) and the backward runs the
adjoint steps on them without recomputing anything (bh_leapfrog_vjp_stored).
The tree's opening decisions are held fixed in every force VJP.
"""
from __future__ import annotations

import torch

from .api import Context


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x0, v0, mass, ctx: Context, dt, nsteps, theta, softening, eps, every,
                keep):
        x = x0.detach().clone()
        v = v0.detach().clone()
        m = mass.detach()
        if theta >= 0:
            a = ctx.compute_accel(x, m, theta, softening=softening, eps=eps, sync=False)
        else:
            a = ctx.compute_accel_direct(x, m, softening=softening, eps=eps, sync=False)
        ckpts = []
        traj = None
        if keep:
            traj = torch.empty((max(nsteps, 1), x.shape[0], 3), dtype=torch.float64,
                               device=x.device)
            for k in range(nsteps):
                ctx.step_leapfrog(x, v, m, a, dt, 1, theta=theta, softening=softening, eps=eps,
                                  sync=False)
                traj[k].copy_(x)
        else:
            done = 0
            while done < nsteps:
                seg = min(every, nsteps - done)
                ckpts.append((x.clone(), v.clone(), a.clone(), seg))
                ctx.step_leapfrog(x, v, m, a, dt, seg, theta=theta, softening=softening, eps=eps,
                                  sync=False)
                done += seg
        ctx.sync()
        fctx.ctx, fctx.ckpts, fctx.traj = ctx, ckpts, traj
        fctx.args = (dt, theta, softening, eps, every, nsteps)
        fctx.save_for_backward(x0.detach(), m)
        return x, v

    @staticmethod
    def backward(fctx, gx, gv):
        x0, m = fctx.saved_tensors
        ctx, ckpts = fctx.ctx, fctx.ckpts
        dt, theta, softening, eps, every, nsteps = fctx.args
        n = x0.shape[0]
        xbar = torch.zeros_like(x0) if gx is None else gx.detach().clone().contiguous()
        vbar = torch.zeros_like(x0) if gv is None else gv.detach().clone().contiguous()
        abar = torch.zeros_like(x0)
        gm = torch.zeros_like(m)
        if fctx.traj is not None:
            ctx.leapfrog_vjp_stored(fctx.traj, m, dt, nsteps, xbar, vbar, abar, gm, theta=theta,
                                    softening=softening, eps=eps, sync=False)
        else:
            traj = torch.empty((max(every, 1), n, 3), dtype=torch.float64, device=x0.device)
            for (x, v, a, seg) in reversed(ckpts):
                ctx.leapfrog_vjp(x, v, a, m, dt, seg, traj, xbar, vbar, abar, gm, theta=theta,
                                 softening=softening, eps=eps, sync=False)
        ctx.accel_vjp(x0.contiguous(), m, abar, theta=theta, softening=softening, eps=eps,
                      g_pos=xbar, g_mass=gm, sync=False)
        ctx.sync()
        return xbar, vbar, gm, None, None, None, None, None, None, None, None


def rollout(x0, v0, mass, ctx: Context, dt: float, nsteps: int, theta: float = 0.5,
            softening: float = 0.0, eps=None, checkpoint_every: int = 20,
            keep_positions: bool = False):
    """(x_T, v_T) after nsteps KDK steps; differentiable in x0, v0 and mass.

    ``ctx`` must be created with ``adjoint=True``. theta < 0 uses the direct sum.
    ``keep_positions`` trades 24 bytes per body and step of device memory for
    a backward pass without recomputation (``checkpoint_every`` is then unused).
    """
    if checkpoint_every < 1:
        raise ValueError("checkpoint_every must be >= 1")
    return _Rollout.apply(x0, v0, mass, ctx, float(dt), int(nsteps), float(theta),
                          float(softening), eps, int(checkpoint_every), bool(keep_positions))
