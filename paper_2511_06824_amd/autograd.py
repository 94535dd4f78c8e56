"""Differentiable force/moment of the piston gap: a torch.autograd.Function whose backward
is the adjoint vector-Jacobian product of the HIP library (one adjoint solve on the
symmetric operator of the base condition)."""

import torch

from . import gapsolve as G


class GapForce(torch.autograd.Function):
    """F = (Fx, Fy, Mx, My)(e, edot) of one working condition.

    forward: assemble the condition, PCG solve, integrate.  backward: re-assemble the saved
    state (the handle may have been used in between) and take w^T dF/d(e, edot) from
    jacobian_adjoint with w = grad_output."""

    @staticmethod
    def forward(ctx, e, edot, solver, opts, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0):
        ev = [float(v) for v in e.detach().cpu().tolist()]
        edv = [float(v) for v in edot.detach().cpu().tolist()]
        solver.assemble(ev, edv, None, 1)
        solver.solve(opts)
        F = solver.integrate(cavitation, p_cav)[0].clone()
        ctx.solver, ctx.opts, ctx.cav, ctx.p_cav = solver, opts, cavitation, p_cav
        ctx.state = (ev, edv)
        ctx.p0 = solver.p[: solver.n].clone()
        ctx.in_device, ctx.in_dtype = e.device, e.dtype
        return F.to(e.device)

    @staticmethod
    def backward(ctx, grad_F):
        solver = ctx.solver
        ev, edv = ctx.state
        solver.assemble(ev, edv, None, 1)
        w = [float(v) for v in grad_F.detach().cpu().tolist()]
        vjp, _ = solver.jacobian_adjoint(ctx.opts, p0=ctx.p0, cavitation=ctx.cav, p_cav=ctx.p_cav, w=w)
        vjp = vjp.to(device=ctx.in_device, dtype=ctx.in_dtype)
        return vjp[:4], vjp[4:], None, None, None, None


def gap_force(e, edot, solver, opts=None, cavitation=G.GAP_CAVITATION_NONE, p_cav=0.0):
    """Differentiable (Fx, Fy, Mx, My) for eccentricities e (4) and rates edot (4), float64."""
    opts = opts if opts is not None else solver.options()
    return GapForce.apply(e, edot, solver, opts, cavitation, p_cav)
