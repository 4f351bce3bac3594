"""torch.autograd.Functions: densities -> compliances, with the hand-written
adjoint, and the density filter (Sec. 2.2, Eqs. (4)-(5)) with its chain rule.

Forward: one FEA + sensitivity step through the C ABI (u, c = f^T u and
g = dc/drho per load case).  Compliance is self-adjoint (the adjoint state is
-u), so g is the whole backward and no second solve is needed; backward
returns sum_l grad_l g_l, combined by a library kernel.
"""

import torch

from . import mto


class MTOCompliance(torch.autograd.Function):
    """c = MTOCompliance.apply(rho, plan): compliances [total load cases] of
    every instance of ``plan`` (layout of mto.h) for densities rho."""

    @staticmethod
    def forward(ctx, rho, plan):
        need_grad = ctx.needs_input_grad[0]
        u, c, g, stats = plan.solve(rho.detach().contiguous(), sensitivities=need_grad)
        ctx.plan = plan
        ctx.stats = stats
        if need_grad:
            ctx.save_for_backward(g)
        return c

    @staticmethod
    def backward(ctx, grad_c):
        (g,) = ctx.saved_tensors
        grad_rho = ctx.plan.weighted_sensitivity(g, grad_c.detach().contiguous().to(torch.float64))
        return grad_rho, None


def total_compliance(rho, plan):
    """Sum of the compliances of all load cases and instances (the objective
    of a multi-load compliance design)."""
    return MTOCompliance.apply(rho, plan).sum()


class MTOMechanism(torch.autograd.Function):
    """J = MTOMechanism.apply(rho, plan, out_index): the compliant-mechanism
    objective of Sec. 4.1, J = z^T u = u[out_index] for a one-instance plan
    whose load case 0 is the input force and load case 1 the unit load at the
    output DOF (out_index is that DOF in the u layout).  Load case 1's
    solution is the adjoint state (K lam = z, K symmetric), so backward is
    dJ/drho = -E'(rho) lam_e^T K_s u_e, from one bilinear sensitivity call."""

    @staticmethod
    def forward(ctx, rho, plan, out_index):
        rho = rho.detach().contiguous()
        u, _, _, stats = plan.solve(rho, sensitivities=False)
        n = plan.instances[0]["n_dof"]
        ctx.plan, ctx.stats = plan, stats
        ctx.save_for_backward(rho, u)
        return u[out_index].clone()

    @staticmethod
    def backward(ctx, grad_J):
        rho, u = ctx.saved_tensors
        plan = ctx.plan
        n = plan.instances[0]["n_dof"]
        lam = torch.cat([u[n:2 * n], u[:n]])  # system 0 pairs with the adjoint state of case 1
        g = plan.adjoint_sensitivity(rho, u, lam)
        return grad_J * g[:plan.instances[0]["n_cells"]], None, None


class DensityFilter(torch.autograd.Function):
    """rho~ = DensityFilter.apply(rho, filt): filtered densities; backward is
    the transposed filter (the chain rule through Eq. (4))."""

    @staticmethod
    def forward(ctx, rho, filt):
        ctx.filt = filt
        return filt.apply(rho.detach().contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        return ctx.filt.grad(grad_out.detach().contiguous().to(torch.float64)), None


def filtered_total_compliance(rho, plan, filt):
    """Sum of all compliances at the filtered densities W rho."""
    return total_compliance(DensityFilter.apply(rho, filt), plan)
