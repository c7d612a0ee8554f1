"""Differentiation form: an implicit simulation as a torch.autograd.Function of
the per-cell log-permeability.

forward runs the implicit steps through nks_newton_step; backward runs the
discrete BDF1/BDF2 adjoint through nks_adjoint (transposed Jacobians with the
transposed Schwarz preconditioner, then (dF/dln K)^T lambda per step).  Both
are library calls; this module only marshals arguments.
"""
from dataclasses import replace

import numpy as np

from . import Grid


def _torch():
    import torch
    return torch


class WellPressureObjective:
    """G(ln K) = sum_i w_i p_i^{n} after n implicit steps (BDF1, then BDF2)
    of one reservoir, as a differentiable function of theta = ln K per cell.

    theta scales all three permeability components of a cell together: the
    template's anisotropy ratios ky/kx and kz/kx are kept.

        obj = WellPressureObjective(problem, settings, nsteps, dt, weights)
        G = obj(theta)            # theta: float64 CUDA tensor of N cells
        G.backward()              # theta.grad = dG/dln K by the adjoint
    """

    def __init__(self, problem, settings, nsteps, dt, weights, adjoint_rtol=1e-10):
        self.problem = problem
        self.settings = settings
        self.nsteps = int(nsteps)
        self.dt = float(dt)
        self.weights = np.asarray(weights, dtype=np.float64)
        self.adjoint_rtol = adjoint_rtol
        kx = np.asarray(problem.kx, dtype=np.float64)
        self.ry = np.asarray(problem.ky, dtype=np.float64) / kx
        self.rz = np.asarray(problem.kz, dtype=np.float64) / kx
        self.last = None
        self._fn = _make_function()

    def problem_at(self, theta):
        k = np.exp(theta.detach().cpu().numpy().astype(np.float64))
        return replace(self.problem, kx=k, ky=k * self.ry, kz=k * self.rz)

    def __call__(self, theta):
        return self._fn.apply(theta, self)


def _make_function():
    torch = _torch()

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, obj):
            grid = Grid([obj.problem_at(theta)], device=theta.device)
            hist, stats = grid.simulate(obj.nsteps, obj.dt, obj.settings)
            G = float(obj.weights @ hist[-1].cpu().numpy())
            ctx.obj, ctx.grid, ctx.hist = obj, grid, hist
            obj.last = dict(stats=stats)
            return torch.tensor(G, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(ctx, gout):
            obj, grid = ctx.obj, ctx.grid
            # the incoming scalar scales the objective's weights, so the
            # adjoint returns the chain-ruled gradient directly
            dG = [None] * (obj.nsteps + 1)
            dG[obj.nsteps] = grid.from_numpy(obj.weights * float(gout))
            grad, st = grid.adjoint(ctx.hist, obj.dt, dG, obj.settings, rtol=obj.adjoint_rtol)
            obj.last["adjoint"] = st
            return grad, None

    return _Fn
