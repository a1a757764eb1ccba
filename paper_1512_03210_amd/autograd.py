"""torch.autograd wrappers of the split step and of <Lz>, on the library's
hand-written adjoint (fse_step_adjoint, fse_apply_Lz).

evolve(plan, psi0, U, nsteps, dt, checkpoint) returns psi after nsteps
TS2-GauSum steps from psi0 at the plan's time, with U (or nothing) as the grid
potential of the step; it is differentiable in psi0 and U.  The forward pass
keeps psi at the start of every segment of `checkpoint` steps; the backward
pass reverses the segments last to first, each call of fse_step_adjoint
recomputing its own forward states from the segment's checkpoint.
The plan is left with U as its grid potential and its time advanced by
nsteps dt, as after the same fse_step calls.
angular_momentum(plan, psi) is <Lz> with the gradient 2 h^d Lz psi (fse_angular_momentum_grad).

Gradients follow torch's convention for complex tensors,
dL/dRe(psi) + i dL/dIm(psi), which is also the library's.
"""
from __future__ import annotations


import torch


class _Evolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, U, plan, nsteps, dt, checkpoint):
        Ud = None if U is None else U.detach().contiguous()
        plan.set_potential(Ud)
        x = psi0.detach().clone().contiguous()
        ckpts = []
        done = 0
        while done < nsteps:
            k = min(int(checkpoint), nsteps - done)
            ckpts.append((plan.time, x.clone(), k))
            plan.step(x, k, dt)
            done += k
        ctx.plan, ctx.dt, ctx.ckpts, ctx.t_end, ctx.U = plan, dt, ckpts, plan.time, Ud
        return x

    @staticmethod
    def backward(ctx, g_out):
        plan = ctx.plan
        plan.set_potential(ctx.U)
        g = g_out.detach().to(plan.cdtype).contiguous().clone()
        gU = None if ctx.U is None else torch.zeros_like(ctx.U)
        for t, x0, k in reversed(ctx.ckpts):
            plan.time = t
            plan.step_adjoint(x0, k, ctx.dt, g, gU)
        plan.time = ctx.t_end
        return g, gU, None, None, None, None


def evolve(plan, psi0, U=None, nsteps=1, dt=1e-3, checkpoint=20):
    """psi(t + nsteps dt) from psi0, differentiable in psi0 and U (adjoint with checkpoints)."""
    if nsteps < 1 or checkpoint < 1:
        raise ValueError("nsteps and checkpoint must be >= 1")
    return _Evolve.apply(psi0, U, plan, int(nsteps), float(dt), int(checkpoint))


class _Lz(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, plan):
        x = psi.detach().contiguous()
        ctx.plan, ctx.psi = plan, x
        return plan.angular_momentum(x).reshape(())

    @staticmethod
    def backward(ctx, g):
        # 2 h^d g Lz psi, computed by the library with g read on the device
        gd = g.detach().to(device=ctx.psi.device, dtype=torch.float64).reshape(1)
        return ctx.plan.angular_momentum_grad(ctx.psi, gd), None


def angular_momentum(plan, psi):
    """<Lz> = h^d sum conj(psi) Lz psi (eq. AME), differentiable in psi."""
    return _Lz.apply(psi, plan)
