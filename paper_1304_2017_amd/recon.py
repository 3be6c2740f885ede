"""Reconstruction built on the HIP operators of `oat.Plan`.

- `Project` / `Backproject`: torch.autograd.Function wrappers whose backward
  passes are the hand-written adjoint kernels (H^T for H and H for H^T).
- `pls_cg`: the penalised least-squares reconstruction of Sec. IV.A,
  Eq. (PLSObjFuncInt), min ||u - H a||^2 + mu R(a), with the quadratic
  smoothness penalty R of Sec. IV.B (squared differences with the previous
  neighbour along each axis), solved by linear conjugate gradients on the
  normal equations (H^T H + mu L^T L) a = H^T u from a = 0, as in the paper.

All operator applications run in the library's kernels on the GPU; the
vector updates are torch device ops, and every inner product and norm of the
CG recursion is accumulated in FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import torch


class Project(torch.autograd.Function):
    """data = H img; the gradient with respect to img is H^T grad."""

    @staticmethod
    def forward(ctx, img, plan):
        ctx.plan = plan
        return plan.project(img.contiguous())

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.backproject(grad.contiguous(), out_dtype=torch.float32), None


class Backproject(torch.autograd.Function):
    """img = H^T data; the gradient with respect to data is H grad."""

    @staticmethod
    def forward(ctx, data, plan):
        ctx.plan = plan
        return plan.backproject(data.contiguous())

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.project(grad.contiguous(), out_dtype=torch.float32), None


def project(img, plan):
    return Project.apply(img, plan)


def backproject(data, plan):
    return Backproject.apply(data, plan)


def smoothness_penalty(a: torch.Tensor) -> torch.Tensor:
    """R(a) = sum_n sum_axes (a_n - a_{n - axis})^2 over pairs inside the grid
    (Sec. IV.B); returned in FP64."""
    a = a.double()
    return ((a[1:] - a[:-1]) ** 2).sum() + ((a[:, 1:] - a[:, :-1]) ** 2).sum() + \
        ((a[:, :, 1:] - a[:, :, :-1]) ** 2).sum()


def smoothness_normal(a: torch.Tensor) -> torch.Tensor:
    """L^T L a for the difference operator L of `smoothness_penalty`
    (the gradient of R is 2 L^T L a)."""
    out = torch.zeros_like(a)
    for dim in range(3):
        d = torch.diff(a, dim=dim)
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[dim] = slice(1, None)
        sl_lo[dim] = slice(None, -1)
        out[tuple(sl_hi)] += d
        out[tuple(sl_lo)] -= d
    return out


def _dot(a: torch.Tensor, b: torch.Tensor) -> float:
    return float(torch.dot(a.reshape(-1).double(), b.reshape(-1).double()))


@dataclass
class PLSResult:
    image: torch.Tensor
    residuals: List[float] = field(default_factory=list)    # ||u - H a_i|| / ||u||
    objective: List[float] = field(default_factory=list)    # ||u - H a_i||^2 + mu R(a_i)


def pls_cg(plan, u: torch.Tensor, mu: float = 0.0, iters: int = 20,
           track: bool = True) -> PLSResult:
    """Linear CG for (H^T H + mu L^T L) a = H^T u, a_0 = 0 (Sec. IV.A-B)."""
    u = u.float().contiguous()
    unorm = max(_dot(u, u) ** 0.5, 1e-300)
    a = torch.zeros(plan.image_shape, device=u.device, dtype=torch.float32)
    r = plan.backproject(u)                         # b - A a_0 with a_0 = 0
    p = r.clone()
    rr = _dot(r, r)
    res = PLSResult(a)
    if track:
        res.residuals.append(1.0)
        res.objective.append(unorm ** 2)
    for _ in range(iters):
        Hp = plan.project(p)
        Ap = plan.backproject(Hp)
        if mu:
            Ap = Ap + mu * smoothness_normal(p)
        pAp = _dot(p, Ap)
        if pAp <= 0.0 or rr == 0.0:
            break
        alpha = rr / pAp
        a = a + alpha * p
        r = r - alpha * Ap
        rr_new = _dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        if track:
            d = u - plan.project(a)
            dn = _dot(d, d)
            res.residuals.append(dn ** 0.5 / unorm)
            res.objective.append(dn + (mu * float(smoothness_penalty(a)) if mu else 0.0))
    res.image = a
    return res
