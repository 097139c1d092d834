"""torch.autograd wrappers of the library's adjoint entry points.

Each Function only marshals tensors to the C ABI: the forward passes run the
library's residual, drag and steady-solve kernels, the backward passes its
transposed-Jacobian kernel and adjoint V-cycle.  The parameter derivatives
of the residual and of the drag at a fixed state (dR/dtheta|_u,
dC_D/dtheta|_u) are central differences over handles built at theta +- h,
formed inside the library (eg_param_sensitivity); everything else is the
discrete adjoint (dR/du)^T lambda + dC_D/du = 0,
dC_D/dtheta = dC_D/dtheta|_u + lambda . dR/dtheta|_u.
"""

from __future__ import annotations

import dataclasses

import torch

from .binding import Solver


class Residual(torch.autograd.Function):
    """R_p(u) (level-p vectors); backward: (dR_p/du)^T grad by the
    transposed-Jacobian kernel at u."""

    @staticmethod
    def forward(ctx, u, solver: Solver, p: int):
        ctx.solver, ctx.p = solver, p
        ctx.save_for_backward(u)
        return solver.residual(p, u.contiguous())

    @staticmethod
    def backward(ctx, grad):
        (u,) = ctx.saved_tensors
        return ctx.solver.adjoint_apply(ctx.p, u.contiguous(), grad.contiguous()), None, None


class Drag(torch.autograd.Function):
    """Pressure drag coefficient of the level-p_max state u; backward:
    grad * dC_D/du."""

    @staticmethod
    def forward(ctx, u, solver: Solver, sref: float = 1.0):
        cd, g = solver.drag(u.contiguous(), sref=sref, grad=True)
        ctx.save_for_backward(g)
        return torch.tensor(cd, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, grad):
        (g,) = ctx.saved_tensors
        return grad * g, None, None


@dataclasses.dataclass
class SteadyDragProblem:
    """C_D of the converged steady state on ``base`` with radial Gaussian wall
    bumps (``wall_bumps(base, amps, centers, sigma)``) as a function of
    theta = (Mach, amp_1, ..., amp_k)."""
    base: object
    centers: object
    sigma: float
    p_max: int
    solver_kw: dict = dataclasses.field(default_factory=dict)
    sref: float = 1.0
    drop: float = 1e-12
    max_cycles: int = 20000
    adjoint_drop: float = 1e-12
    adjoint_max_cycles: int = 20000
    fd_step: float = 1e-6

    def solver(self, theta):
        from eg_inputs import wall_bumps
        th = [float(x) for x in theta]
        mesh = wall_bumps(self.base, th[1:], self.centers, self.sigma) if len(th) > 1 else self.base
        return Solver(mesh, self.p_max, mach=th[0], **self.solver_kw)

    def steady(self, S: Solver, u=None):
        u = S.freestream(self.p_max) if u is None else u
        _, st = S.solve_steady(u, drop_tol=self.drop, max_cycles=self.max_cycles, raise_on_fail=True)
        return u


class SteadyDrag(torch.autograd.Function):
    """theta (float64 tensor [1 + k]: Mach, bump amplitudes) -> C_D of the
    converged steady state; backward by the discrete adjoint."""

    @staticmethod
    def forward(ctx, theta, prob: SteadyDragProblem):
        S = prob.solver(theta.tolist())
        u = prob.steady(S)
        cd = S.drag(u, sref=prob.sref)
        ctx.prob, ctx.S, ctx.u = prob, S, u
        ctx.theta = theta.detach().cpu().tolist()
        return torch.tensor(cd, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad):
        prob, S, u, th = ctx.prob, ctx.S, ctx.u, ctx.theta
        _, g = S.drag(u, sref=prob.sref, grad=True)
        lam, _, _ = S.adjoint_solve(u, g, drop_tol=prob.adjoint_drop, max_cycles=prob.adjoint_max_cycles)
        h = prob.fd_step
        out = torch.zeros(len(th), dtype=torch.float64)
        direction = None
        for i in range(len(th)):
            tp, tm = list(th), list(th)
            tp[i] += h
            tm[i] -= h
            Sp, Sm = prob.solver(tp), prob.solver(tm)
            if direction is None:
                from .binding import _freestream_direction
                direction = _freestream_direction(S.dim, S.alpha_deg, S.beta_deg)
            out[i] = Sp.param_sensitivity(Sm, h, u, lam, direction=direction, sref=prob.sref)
            Sp.close()
            Sm.close()
        return grad * out, None
