"""Differentiable traveltime operator and TV-regularised inversion.

``apply_J(op, dc)`` is the forward operator dT = J dc (paper Sec. II-C,
eq. forward_compact) as a torch autograd function whose backward is the
library's J^T kernel, so nonlinear regularisers can be optimised through it.
``misfit_tv`` is the objective of eq. leastSquare_misfit1 with Gamma_n =
sigma^2 I and a smoothed isotropic total-variation term (the regulariser the
paper uses for its reconstructions, Sec. III), and ``invert_tv`` minimises it
with torch's L-BFGS.
"""
from __future__ import annotations

import torch

from . import fftt


class _ApplyJ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dc, op, prec):
        ctx.op = op
        ctx.prec = prec
        return op.apply_J(dc.detach().contiguous(), prec=prec)

    @staticmethod
    def backward(ctx, g):
        return ctx.op.apply_JT(g.detach().contiguous(), prec=ctx.prec), None, None


def apply_J(op: "fftt.Context", dc: torch.Tensor, prec: int = fftt.FP32) -> torch.Tensor:
    """J dc for every band ([B*M]); differentiable in dc."""
    return _ApplyJ.apply(dc, op, prec)


def tv(x: torch.Tensor, dims, spacing, beta: float) -> torch.Tensor:
    """sum_j sqrt(|grad x|_j^2 + beta^2): forward differences scaled by 1/h,
    zero difference at the upper boundary of each axis (x fastest)."""
    nx, ny, nz = dims
    u = x.reshape(nz, ny, nx)
    dx = torch.zeros_like(u)
    dy = torch.zeros_like(u)
    dz = torch.zeros_like(u)
    dx[:, :, :-1] = (u[:, :, 1:] - u[:, :, :-1]) / spacing[0]
    dy[:, :-1, :] = (u[:, 1:, :] - u[:, :-1, :]) / spacing[1]
    dz[:-1, :, :] = (u[1:, :, :] - u[:-1, :, :]) / spacing[2]
    return torch.sqrt(dx * dx + dy * dy + dz * dz + beta * beta).sum()


def misfit_tv(op, x, d_obs, sigma, alpha_tv, beta, dims, spacing, prec=fftt.FP32):
    """1/2 |J x - d|^2 / sigma^2 + alpha_tv TV_beta(x), all bands."""
    r = apply_J(op, x, prec) - d_obs
    return 0.5 * (r * r).sum() / sigma ** 2 + alpha_tv * tv(x, dims, spacing, beta)


def invert_tv(op, d_obs, sigma, alpha_tv, beta, dims, spacing, iters=20, prec=fftt.FP32,
              x0=None, history_size=10, max_eval=None):
    """Minimise misfit_tv with L-BFGS (strong Wolfe line search): at most
    `iters` iterations and `max_eval` objective evaluations (default 1.25
    iters, the optimizer's own); returns (x, list of objective values per
    evaluation)."""
    dt = torch.float64 if prec == fftt.FP64 else torch.float32
    n = int(dims[0] * dims[1] * dims[2])
    x = (torch.zeros(n, dtype=dt, device=d_obs.device) if x0 is None
         else x0.detach().clone().to(dt))
    x.requires_grad_(True)
    opt = torch.optim.LBFGS([x], lr=1.0, max_iter=iters, max_eval=max_eval,
                            history_size=history_size, line_search_fn="strong_wolfe",
                            tolerance_grad=0.0, tolerance_change=0.0)
    hist = []

    def closure():
        opt.zero_grad()
        f = misfit_tv(op, x, d_obs, sigma, alpha_tv, beta, dims, spacing, prec)
        f.backward()
        hist.append(float(f.detach()))
        return f

    opt.step(closure)
    return x.detach(), hist
