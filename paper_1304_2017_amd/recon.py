"""Reconstruction built on the HIP operators of `oat.Plan`.

- `Project` / `Backproject`: torch.autograd.Function wrappers whose backward
  passes are the hand-written adjoint kernels (H^T for H and H for H^T).
- `pls_cg`: the penalised least-squares reconstruction of Sec. IV.A,
  Eq. (PLSObjFuncInt), min ||u - H a||^2 + mu R(a), with the quadratic
  smoothness penalty R of Sec. IV.B (squared differences with the previous
  neighbour along each axis), solved by linear conjugate gradients on the
  normal equations (H^T H + mu L^T L) a = H^T u from a = 0, as in the paper.
- `pls_tv`: the same data term with a smoothed isotropic total-variation
  penalty TV_eps(a) = sum_n sqrt(|grad a|_n^2 + eps^2) (forward differences,
  zero across the far faces) instead of R.  The paper has no TV penalty;
  this is the usual smoothed form.  Nonlinear conjugate gradients
  (Polak-Ribiere+, restarted when not a descent direction) with a
  majorise-minimise step: along a direction d the data term is an exact
  quadratic and TV_eps lies below the quadratic obtained from
  sqrt(x) <= sqrt(x0) + (x - x0) / (2 sqrt(x0)), so the step that minimises
  the sum decreases the objective at every iteration.  One H and one H^T
  per iteration.

All operator applications run in the library's kernels on the GPU; the
vector updates are torch device ops, and every inner product and norm of the
CG recursion is accumulated in FP64.
"""
from __future__ import annotations

import time
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
    times: List[float] = field(default_factory=list)        # wall seconds to a_i (device synced)


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


def forward_diff(a: torch.Tensor):
    """(d_x, d_y, d_z) with d_x[z, y, x] = a[z, y, x+1] - a[z, y, x] and 0 in
    the last slice of each axis."""
    d = []
    for dim in (2, 1, 0):
        g = torch.zeros_like(a)
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[dim] = slice(1, None)
        lo[dim] = slice(None, -1)
        g[tuple(lo)] = a[tuple(hi)] - a[tuple(lo)]
        d.append(g)
    return d


def forward_diff_adj(gx: torch.Tensor, gy: torch.Tensor, gz: torch.Tensor) -> torch.Tensor:
    """Adjoint of `forward_diff` (a negative divergence)."""
    out = torch.zeros_like(gx)
    for g, dim in ((gx, 2), (gy, 1), (gz, 0)):
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[dim] = slice(1, None)
        lo[dim] = slice(None, -1)
        inner = g[tuple(lo)]
        out[tuple(hi)] += inner
        out[tuple(lo)] -= inner
    return out


def tv_eps(a: torch.Tensor, eps: float):
    """(TV_eps(a) in FP64, its gradient, the weights 1/sqrt(|grad a|^2 + eps^2))."""
    gx, gy, gz = forward_diff(a)
    s = torch.sqrt(gx * gx + gy * gy + gz * gz + eps * eps)
    w = 1.0 / s
    grad = forward_diff_adj(gx * w, gy * w, gz * w)
    return float(s.double().sum()), grad, w


def _pls_tv_steps(plan, u: torch.Tensor, mu: float, eps: float, iters: int, storage):
    """The PLS-TV recursion; yields (a, g, ||u - H a||^2, TV_eps(a)) for the
    start a = 0 and after every iteration."""
    def H(x):
        return plan.project(x.to(storage).contiguous(), out_dtype=storage).float()

    def HT(y):
        return plan.backproject(y.to(storage).contiguous(), out_dtype=storage).float()

    a = torch.zeros(plan.image_shape, device=u.device, dtype=torch.float32)
    r = u.clone()                                    # u - H a
    tv, tg, w = tv_eps(a, eps)
    g = -2.0 * HT(r) + mu * tg
    d = -g
    yield a, g, _dot(r, r), tv
    gg = _dot(g, g)
    for _ in range(iters):
        Hd = H(d)
        dx, dy, dz = forward_diff(d)
        curv = float((w.double() * (dx * dx + dy * dy + dz * dz).double()).sum())
        den = 2.0 * _dot(Hd, Hd) + mu * curv
        slope = _dot(g, d)
        if den <= 0.0 or slope >= 0.0:
            return
        t = -slope / den
        a = a + t * d
        r = r - t * Hd
        tv, tg, w = tv_eps(a, eps)
        g_new = -2.0 * HT(r) + mu * tg
        gg_new = _dot(g_new, g_new)
        beta = max(0.0, (gg_new - _dot(g_new, g)) / gg) if gg > 0 else 0.0
        d = -g_new + beta * d
        if _dot(g_new, d) >= 0.0:
            d = -g_new
        g, gg = g_new, gg_new
        yield a, g, _dot(r, r), tv


def pls_tv(plan, u: torch.Tensor, mu: float, eps: float, iters: int = 20,
           storage=torch.float32, track: bool = True) -> PLSResult:
    """Nonlinear CG for min ||u - H a||^2 + mu TV_eps(a) from a = 0.
    `storage` is the dtype of the operator inputs and outputs (FP32 or BF16);
    iterates and residuals are kept in FP32 and every inner product in FP64."""
    t0 = time.perf_counter()
    u = u.float().contiguous()
    unorm = max(_dot(u, u) ** 0.5, 1e-300)
    res = PLSResult(None)
    for a, _, rn, tv in _pls_tv_steps(plan, u, mu, eps, iters, storage):
        res.image = a
        if track:
            res.residuals.append(rn ** 0.5 / unorm)
            res.objective.append(rn + mu * tv)
            res.times.append(time.perf_counter() - t0)   # rn is an FP64 dot: the device is synced
    return res


def pls_tv_iterates(plan, u: torch.Tensor, mu: float, eps: float, iters: int = 10,
                    storage=torch.float32):
    """(a_k, g_k) for k = 0 .. iters-1 of `pls_tv` (iterate and objective
    gradient before step k)."""
    u = u.float().contiguous()
    for k, (a, g, _, _) in enumerate(_pls_tv_steps(plan, u, mu, eps, iters - 1, storage)):
        yield a, g
