"""torch.autograd wrapper of the state solve.

forward:  x (raw design, [E]) -> s ([N][5]): filter, RAMP and the Newton state solve.
backward: grad_s -> grad_x: the adjoint solve J~^T lambda = grad_s at the converged
state and the sensitivities -lambda^T dR/dgamma pulled back through RAMP and the
filter transpose (Sec. 5.1, adjoint sensitivity analysis).  Both directions run in the
HIP library; the objective f = f_qh^T t is an ordinary torch product on s, so any
differentiable function of the state can be used as the loss.
"""

import torch

from . import nc


class StateSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, solver, s0=None):
        x = x.detach()
        solver.set_design(x)
        s = solver.solve_state(s0=s0)
        if solver.last_info["status"] != nc.NC_OK:
            raise RuntimeError(f"state solve did not converge: {solver.last_info}")
        ctx.solver = solver
        ctx.save_for_backward(x, s)
        return s

    @staticmethod
    def backward(ctx, grad_s):
        x, s = ctx.saved_tensors
        solver = ctx.solver
        solver.set_design(x)   # the context may have been given another design since forward
        lam = solver.solve_adjoint(s, grad_s.contiguous().to(torch.float64))
        if solver.last_info["status"] != nc.NC_OK:
            raise RuntimeError(f"adjoint solve did not converge: {solver.last_info}")
        dfdx = solver.sensitivity(s, lam)
        return dfdx.to(x.dtype), None, None


def solve_state(x, solver, s0=None):
    """Differentiable state solve: returns s with s.grad_fn tied to the adjoint."""
    return StateSolve.apply(x, solver, s0)


def compliance(s, solver):
    """Thermal compliance f = f_qh^T t with the boundary-flux load (differentiable in s)."""
    g = solver.objective_grad()
    return (s * g).sum()
