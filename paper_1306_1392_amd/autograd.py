"""Adjoint autograd pairs over the HIP projector and backprojector.

Project(x) = A x with A = s^2 B^T (forward_project); its backward is A^T g =
s^2 B g (backproject with alpha = s^2).  BackProject(q) = B q; its backward is
B^T g = A g / s^2 (forward_project with alpha = 1/s^2).  FBP(p) = B(F p) with F
the row-weighted ramp filter; its backward is F^T (B^T g), and F^T = F for
full-detector scans: the Ram-Lak kernel is even, so the convolution on [0, L)
is a symmetric matrix, and each row's quadrature weight is one scalar, which
commutes with it.  No extra kernel exists for the backward passes: each is the
adjoint call, and every product runs in the library."""
from __future__ import annotations

import torch

from . import api


def _s2(plan: api.Plan) -> float:
    return float(plan.geom0.pixel_size) ** 2


class Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return api.forward_project(plan, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        return api.backproject(plan, g.contiguous(), 0, alpha=_s2(plan)), None


class BackProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, plan):
        ctx.plan = plan
        return api.backproject(plan, q.contiguous(), 0)

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        return api.forward_project(plan, g.contiguous(), alpha=1.0 / _s2(plan)), None


class FBP(torch.autograd.Function):
    """Filtered backprojection of line integrals (full-detector scans)."""

    @staticmethod
    def forward(ctx, p, plan):
        for g in plan.geoms:
            if g.scan == api.SCAN_360_HALF:
                raise ValueError("FBP autograd: half-acquisition rows are extended; use fbp_filter/backproject")
        ctx.plan = plan
        return api.backproject(plan, api.fbp_filter(plan, p.contiguous()), 1)

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        bt = api.forward_project(plan, g.contiguous(), alpha=1.0 / _s2(plan))
        return api.fbp_filter(plan, bt), None


def project(x, plan):
    return Project.apply(x, plan)


def backproject(q, plan):
    return BackProject.apply(q, plan)


def fbp(p, plan):
    return FBP.apply(p, plan)
