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

Both solvers can write their state every few iterations (`checkpoint`,
`every`) and continue from such a file (`resume`); the continued run takes
exactly the steps of an uninterrupted one.  `rmse` is the accuracy measure
of Sec. IV.A.
"""
from __future__ import annotations

import os
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

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


def rmse(a: torch.Tensor, ref) -> float:
    """Root mean square error of Sec. IV.A, sqrt((a - ref)^T (a - ref) / N),
    accumulated in FP64 (ref: tensor or array of the same shape)."""
    r = torch.as_tensor(ref, device=a.device).double()
    d = a.double() - r
    return float(torch.sqrt(torch.dot(d.reshape(-1), d.reshape(-1)) / d.numel()))


def save_state(path: str, state: dict) -> None:
    """Write a solver state (tensors, numbers, lists of numbers) with
    torch.save, tensors on the CPU; written to a temporary file and renamed,
    so a reader never sees a partial file."""
    cpu = {k: (v.detach().cpu() if isinstance(v, torch.Tensor) else v) for k, v in state.items()}
    tmp = path + ".tmp"
    torch.save(cpu, tmp)
    os.replace(tmp, path)


def load_state(path: str, device) -> dict:
    """Read a state written by save_state (weights_only: plain data only),
    tensors moved to `device`."""
    st = torch.load(path, map_location="cpu", weights_only=True)
    return {k: (v.to(device) if isinstance(v, torch.Tensor) else v) for k, v in st.items()}


@dataclass
class PLSResult:
    image: torch.Tensor
    residuals: List[float] = field(default_factory=list)    # ||u - H a_i|| / ||u||
    objective: List[float] = field(default_factory=list)    # ||u - H a_i||^2 + mu R(a_i)
    times: List[float] = field(default_factory=list)        # wall seconds to a_i (device synced)
    directions: List[tuple] = field(default_factory=list)   # learned PLS-TV: (kind, cosine) per step


def pls_cg(plan, u: torch.Tensor, mu: float = 0.0, iters: int = 20, track: bool = True,
           storage=torch.float32, checkpoint: Optional[str] = None, every: int = 0,
           resume: Optional[str] = None) -> PLSResult:
    """Linear CG for (H^T H + mu L^T L) a = H^T u, a_0 = 0 (Sec. IV.A-B).
    One H and one H^T per iteration: the data residual u - H a is updated
    with the H p of each step.  `storage` is the dtype of the operator inputs
    and outputs (FP32 or BF16).  With `checkpoint` and `every` > 0 the state
    is saved after every `every`-th iteration; `resume` continues from such a
    file up to `iters` iterations in all."""
    t0 = time.perf_counter()

    def H(x):
        return plan.project(x.to(storage).contiguous(), out_dtype=storage).float()

    def HT(y):
        return plan.backproject(y.to(storage).contiguous(), out_dtype=storage).float()

    u = u.float().contiguous()
    unorm = max(_dot(u, u) ** 0.5, 1e-300)
    res = PLSResult(None)
    if resume:
        st = load_state(resume, u.device)
        k0, a, r, p, s, rr = st["k"], st["a"], st["r"], st["p"], st["s"], st["rr"]
        res.residuals, res.objective = list(st["residuals"]), list(st["objective"])
        res.times = list(st["times"])
        t0 -= res.times[-1] if res.times else 0.0
    else:
        k0 = 0
        a = torch.zeros(plan.image_shape, device=u.device, dtype=torch.float32)
        r = HT(u)                                     # b - A a_0 with a_0 = 0
        p = r.clone()
        s = u.clone()                                 # u - H a
        rr = _dot(r, r)
        if track:
            res.residuals.append(1.0)
            res.objective.append(unorm ** 2)
            res.times.append(time.perf_counter() - t0)
    for k in range(k0, iters):
        Hp = H(p)
        Ap = HT(Hp)
        if mu:
            Ap = Ap + mu * smoothness_normal(p)
        pAp = _dot(p, Ap)
        if pAp <= 0.0 or rr == 0.0:
            break
        alpha = rr / pAp
        a = a + alpha * p
        s = s - alpha * Hp
        r = r - alpha * Ap
        rr_new = _dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        if track:
            dn = _dot(s, s)
            res.residuals.append(dn ** 0.5 / unorm)
            res.objective.append(dn + (mu * float(smoothness_penalty(a)) if mu else 0.0))
            res.times.append(time.perf_counter() - t0)
        if checkpoint and every > 0 and (k + 1) % every == 0:
            save_state(checkpoint, dict(k=k + 1, a=a, r=r, p=p, s=s, rr=rr,
                                        residuals=res.residuals, objective=res.objective,
                                        times=res.times))
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


def _pls_tv_steps(plan, u: torch.Tensor, mu: float, eps: float, iters: int, storage,
                  state: Optional[dict] = None):
    """The PLS-TV recursion; yields (k, a, g, d, r, gg, ||u - H a||^2, TV_eps(a))
    for the start a = 0 (k = 0) and after every iteration k.  `state` (from a
    checkpoint: k, a, r, g, d, gg) continues a run after its iteration k."""
    def H(x):
        return plan.project(x.to(storage).contiguous(), out_dtype=storage).float()

    def HT(y):
        return plan.backproject(y.to(storage).contiguous(), out_dtype=storage).float()

    if state is None:
        k0 = 0
        a = torch.zeros(plan.image_shape, device=u.device, dtype=torch.float32)
        r = u.clone()                                # u - H a
        tv, tg, w = tv_eps(a, eps)
        g = -2.0 * HT(r) + mu * tg
        d = -g
        gg = _dot(g, g)
        yield 0, a, g, d, r, gg, _dot(r, r), tv
    else:
        k0, a, r, g, d, gg = state["k"], state["a"], state["r"], state["g"], state["d"], state["gg"]
        tv, tg, w = tv_eps(a, eps)
    for k in range(k0, iters):
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
        yield k + 1, a, g, d, r, gg, _dot(r, r), tv


def pls_tv(plan, u: torch.Tensor, mu: float, eps: float, iters: int = 20,
           storage=torch.float32, track: bool = True, checkpoint: Optional[str] = None,
           every: int = 0, resume: Optional[str] = None,
           observe: Optional[Callable[[int, torch.Tensor], None]] = None) -> PLSResult:
    """Nonlinear CG for min ||u - H a||^2 + mu TV_eps(a) from a = 0.
    `storage` is the dtype of the operator inputs and outputs (FP32 or BF16);
    iterates and residuals are kept in FP32 and every inner product in FP64.
    With `checkpoint` and `every` > 0 the state is saved after every
    `every`-th iteration; `resume` continues from such a file up to `iters`
    iterations in all.  `observe(k, a)` is called with every iterate; the
    recorded times leave out its calls."""
    t0 = time.perf_counter()
    u = u.float().contiguous()
    unorm = max(_dot(u, u) ** 0.5, 1e-300)
    res = PLSResult(None)
    state = None
    if resume:
        state = load_state(resume, u.device)
        res.residuals, res.objective = list(state["residuals"]), list(state["objective"])
        res.times = list(state["times"])
        res.image = state["a"]
        t0 -= res.times[-1] if res.times else 0.0
    for k, a, g, d, r, gg, rn, tv in _pls_tv_steps(plan, u, mu, eps, iters, storage, state):
        res.image = a
        if track:
            res.residuals.append(rn ** 0.5 / unorm)
            res.objective.append(rn + mu * tv)
            res.times.append(time.perf_counter() - t0)   # rn is an FP64 dot: the device is synced
        if observe is not None:                       # not counted in the times
            t_obs = time.perf_counter()
            observe(k, a)
            t0 += time.perf_counter() - t_obs
        if checkpoint and every > 0 and k > 0 and k % every == 0:
            save_state(checkpoint, dict(k=k, a=a, r=r, g=g, d=d, gg=gg, residuals=res.residuals,
                                        objective=res.objective, times=res.times))
    return res


def pls_tv_iterates(plan, u: torch.Tensor, mu: float, eps: float, iters: int = 10,
                    storage=torch.float32):
    """(a_k, g_k) for k = 0 .. iters-1 of `pls_tv` (iterate and objective
    gradient before step k)."""
    u = u.float().contiguous()
    for _, a, g, _, _, _, _, _ in _pls_tv_steps(plan, u, mu, eps, iters - 1, storage):
        yield a, g
