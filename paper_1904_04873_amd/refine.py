"""Differentiable stage 2: the bin-interpolated power as a torch.autograd.Function and a
gradient refinement of candidates (an extension of the power statistic of eq:hough3).

The forward is ``bsh_power_stat`` in mode 1, the backward ``bsh_power_stat_grad``; both run in
the library's HIP kernels.  The refinement loop can take both from one pass
(``bsh_power_stat_value_and_grad``).  P_lin is piecewise linear in the parameters, with kinks where a
track crosses a bin edge; the backward returns the right-hand derivative there.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import bsh


class BshPower(torch.autograd.Function):
    """P_lin(theta) for candidates theta = (F = f0 Tc, a_p, P, t_asc) [n, 4] float64."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, seg: "bsh.DeviceSegments", sky: torch.Tensor,
                cand_sky: torch.Tensor, status: Optional["bsh.Status"] = None):
        theta = theta.detach().contiguous()
        P = bsh.bsh_power_stat(seg, sky, cand_sky, theta, mode=1, status=status)
        ctx.save_for_backward(theta)
        ctx.seg, ctx.sky, ctx.cand_sky, ctx.status = seg, sky, cand_sky, status
        return P.to(torch.float64)

    @staticmethod
    def backward(ctx, grad_P: torch.Tensor):
        (theta,) = ctx.saved_tensors
        g = bsh.bsh_power_stat_grad(ctx.seg, ctx.sky, ctx.cand_sky, theta,
                                    grad_P.to(torch.float64).contiguous(), status=ctx.status)
        return g, None, None, None, None


def power_lin(theta, seg, sky, cand_sky, status=None) -> torch.Tensor:
    return BshPower.apply(theta, seg, sky, cand_sky, status)


def refine(theta0: torch.Tensor, steps: torch.Tensor, seg, sky, cand_sky, n_iter: int = 20,
           lr: float = 0.05, betas=(0.9, 0.999), status=None, fused: bool = True):
    """Adam ascent of P_lin per candidate, in grid-step units u: theta = theta0 + u * steps.

    Candidates are independent (the objective is the sum of their powers, whose gradient
    separates).  With ``fused`` each step takes P_lin and its gradient from one pass of
    ``bsh_power_stat_value_and_grad`` (the same gradient, bit for bit, as the autograd route
    through BshPower, so the same iterates); otherwise it runs the forward and the backward of
    BshPower.  Returns (theta, P_lin history [n_iter + 1, n])."""
    u = torch.zeros_like(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([u], lr=lr, betas=betas)
    hist = []
    for _ in range(n_iter):
        opt.zero_grad(set_to_none=True)
        if fused:
            with torch.no_grad():
                theta = (theta0 + u * steps).contiguous()
                P, g = bsh.bsh_power_stat_value_and_grad(seg, sky, cand_sky, theta, status=status)
                # d(-sum P)/du = -(dP/dtheta) * steps
                u.grad = -(g * steps)
            hist.append(P.to(torch.float64))
        else:
            P = power_lin(theta0 + u * steps, seg, sky, cand_sky, status)
            hist.append(P.detach())
            (-P.sum()).backward()
        opt.step()
    with torch.no_grad():
        theta = theta0 + u * steps
        hist.append(power_lin(theta, seg, sky, cand_sky, status).detach())
    return theta.detach(), torch.stack(hist)
