"""Differentiable pressure solve.

``pressure(theta, problem)`` returns the cell pressures of the MHFE-FV system assembled
with K^E scaled by exp(theta_E), solved by EDFA-preconditioned GMRES on the device.  Its
backward pass solves the transposed system A^T lambda = dL/du with the transposed EDFA
(the forward preconditioner applied as P^-T) and evaluates dL/dtheta_E per cell on the
device (``edfa_grad_logk``).  The derivation: W^E scales as exp(theta_E), so with
R(u; theta) = A(theta) u - b(theta) (eq. system), dL/dtheta = -lambda^T dR/dtheta.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import edfa


class PressureSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, problem, params, rtol, rtol_adjoint, restart):
        mult = np.exp(theta.detach().to("cpu", torch.float64).numpy())
        prob = dataclasses.replace(problem, K=np.asarray(problem.K) * mult[:, None])
        S = edfa.System(prob)
        P = edfa.Precond(S, params)
        flexible = params.precision == 1
        u, info, st = edfa.solve(S, P, S.rhs(), rtol=rtol, restart=restart, flexible=flexible)
        if st != edfa.OK:
            raise RuntimeError(f"forward solve did not converge ({info['iterations']} iterations, "
                               f"relres {info['relres_true']:.3e})")
        ctx.S, ctx.P = S, P
        ctx.opts = (rtol_adjoint, restart, flexible)
        ctx.theta_device = theta.device
        ctx.save_for_backward(u)
        return u[S.info["nfu"]:].clone()

    @staticmethod
    def backward(ctx, gp):
        (u,) = ctx.saved_tensors
        S, P = ctx.S, ctx.P
        rtol_adjoint, restart, flexible = ctx.opts
        nfu = S.info["nfu"]
        rhs = torch.zeros_like(u)
        rhs[nfu:] = gp.to(u.device, torch.float64)
        if not bool(torch.any(rhs != 0)):
            g = torch.zeros(S.info["ne"], dtype=torch.float64, device=u.device)
        else:
            lam, info, st = edfa.solve(S, P, rhs, rtol=rtol_adjoint, restart=restart,
                                       flexible=flexible, transpose=True)
            if st != edfa.OK:
                raise RuntimeError(f"adjoint solve did not converge ({info['iterations']} "
                                   f"iterations, relres {info['relres_true']:.3e})")
            g = edfa.grad_logk(S, u, lam)
        return g.to(ctx.theta_device), None, None, None, None, None


def pressure(theta, problem, params=None, rtol=1e-8, rtol_adjoint=1e-10, restart=50):
    """Cell pressures for permeabilities K^E exp(theta_E); differentiable in theta."""
    if params is None:
        params = edfa.Params("dynamic", n_add=1, n_ent=4)
    return PressureSolve.apply(theta, problem, params, rtol, rtol_adjoint, restart)
