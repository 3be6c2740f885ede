"""Learned preconditioner for the PLS-TV reconstruction (not in the paper).

A three-layer 3-D convolution network, 3x3x3 kernels with 16 channels,
    z = x + C3(relu(C2(relu(C1(x))))),
maps the normalised steepest-descent direction x = -g / rms(g) of the PLS-TV
objective to a search direction z.  The skip connection makes the untrained
network the identity (plain steepest descent).  Inference and training run in
the library's kernels (include/oat_cnn.h): convolutions with FP32 or BF16
activations and FP32 accumulation, the weight gradients, the loss and Adam.
This module only marshals tensors and orders the calls.

`pls_tv_learned` is the PLS-TV iteration of `recon.pls_tv` with z in place of
-g (preconditioned Polak-Ribiere+ conjugacy) and the same majorise-minimise
step; whenever z is not a descent direction the step falls back to -g, so the
objective still decreases at every iteration.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import torch

from . import oat, recon

_DT = {torch.float32: oat.OAT_F32, torch.bfloat16: oat.OAT_BF16}


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def conv3d(x: torch.Tensor, weight: torch.Tensor, bias: Optional[torch.Tensor], relu: bool = False,
           mask: Optional[torch.Tensor] = None, out_dtype=None) -> torch.Tensor:
    """'Same' 3x3x3 convolution of x [C_in, D, H, W] with weight
    [C_out, C_in, 27] (FP32) in the library kernel; optional ReLU and output
    mask (zero where mask <= 0; mask has the output's shape and dtype)."""
    ci, d, h, w = x.shape
    co = weight.shape[0]
    out_dtype = out_dtype or x.dtype
    if tuple(weight.shape) != (co, ci, 27) or weight.dtype != torch.float32:
        raise ValueError(f"weight must be float32 [{co}, {ci}, 27], got {weight.dtype} {tuple(weight.shape)}")
    if bias is not None and (tuple(bias.shape) != (co,) or bias.dtype != torch.float32):
        raise ValueError(f"bias must be float32 [{co}]")
    y = torch.empty((co, d, h, w), device=x.device, dtype=out_dtype)
    if mask is not None and (mask.shape != y.shape or mask.dtype != out_dtype
                             or not mask.is_contiguous()):
        raise ValueError("mask must be contiguous with the output's shape and dtype")
    # the contiguous operands stay referenced until the launch is queued
    xc, wc = x.contiguous(), weight.contiguous()
    bc = bias.contiguous() if bias is not None else None
    oat._check(oat.lib().oat_conv3d_forward(
        _ptr(xc), _DT[x.dtype], ci, d, h, w, _ptr(wc),
        _ptr(bc), co, _ptr(y), _DT[out_dtype], int(relu), _ptr(mask), _stream()))
    return y


def conv3d_weight_grad(x: torch.Tensor, dy: torch.Tensor):
    """(dweight [C_out, C_in, 27], dbias [C_out]) of conv3d for input x and
    output gradient dy, in the library kernel (deterministic tile sums)."""
    ci, d, h, w = x.shape
    co = dy.shape[0]
    L = oat.lib()
    ws = L.oat_conv3d_backward_weight_workspace(ci, co, d, h, w)
    work = torch.empty(max(ws // 4, 1), device=x.device, dtype=torch.float32)
    dw = torch.empty((co, ci, 27), device=x.device, dtype=torch.float32)
    db = torch.empty((co,), device=x.device, dtype=torch.float32)
    if tuple(dy.shape) != (co, d, h, w):
        raise ValueError(f"dy must have shape {(co, d, h, w)}, got {tuple(dy.shape)}")
    xc, dyc = x.contiguous(), dy.contiguous()
    oat._check(L.oat_conv3d_backward_weight(
        _ptr(xc), _DT[x.dtype], _ptr(dyc), _DT[dy.dtype], ci, co, d, h, w,
        _ptr(dw), _ptr(db), _ptr(work), ws, _stream()))
    return dw, db


def flip_transpose(weight: torch.Tensor) -> torch.Tensor:
    """Weights of the adjoint convolution: [C_in, C_out, 27] with the taps
    reversed (tap t -> 26 - t mirrors all three axes)."""
    return weight.transpose(0, 1).flip(2).contiguous()


def mse(y: torch.Tensor, target: torch.Tensor):
    """(loss as a device scalar, dloss/dy) in the library kernel."""
    L = oat.lib()
    if y.shape != target.shape:
        raise ValueError(f"mse: shapes {tuple(y.shape)} and {tuple(target.shape)} differ")
    loss = torch.empty((1,), device=y.device, dtype=torch.float32)
    dy = torch.empty(y.shape, device=y.device, dtype=y.dtype)
    work = torch.empty(L.oat_mse_workspace() // 4, device=y.device, dtype=torch.float32)
    yc, tc = y.contiguous(), target.contiguous()
    oat._check(L.oat_mse(_ptr(yc), _DT[y.dtype], _ptr(tc),
                         _DT[target.dtype], y.numel(), _ptr(loss), _ptr(dy), _ptr(work), _stream()))
    return loss, dy


class Preconditioner:
    """z = x + C3(relu(C2(relu(C1(x))))) with 16 channels and 3x3x3 kernels."""

    CH = 16

    def __init__(self, device=0, seed: int = 0, storage=torch.bfloat16, init_scale: float = 0.1):
        g = torch.Generator().manual_seed(seed)
        dev = torch.device("cuda", device)
        shapes = [(self.CH, 1), (self.CH, self.CH), (1, self.CH)]
        self.w, self.b = [], []
        for li, (co, ci) in enumerate(shapes):
            std = math.sqrt(2.0 / (27 * ci))          # He initialisation for the ReLU layers
            if li == 2:
                std *= init_scale                     # start close to the identity map
            self.w.append((torch.randn((co, ci, 27), generator=g) * std).to(dev))
            self.b.append(torch.zeros((co,), device=dev))
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.step = 0
        self.storage = storage
        self._cache = None

    def parameters(self) -> List[torch.Tensor]:
        return self.w + self.b

    def forward(self, x: torch.Tensor, keep: bool = False) -> torch.Tensor:
        """x: [D, H, W] -> z, same shape, in the storage dtype."""
        x1 = x.to(self.storage).contiguous()[None]
        a1 = conv3d(x1, self.w[0], self.b[0], relu=True)
        a2 = conv3d(a1, self.w[1], self.b[1], relu=True)
        r = conv3d(a2, self.w[2], self.b[2])
        z = (x1.float() + r.float()).to(self.storage)
        if keep:
            self._cache = (x1, a1, a2)
        return z[0]

    def backward(self, dz: torch.Tensor):
        """Parameter gradients for dloss/dz (the last forward had keep=True)."""
        x1, a1, a2 = self._cache
        d3 = dz.to(self.storage).contiguous()[None]
        dw3, db3 = conv3d_weight_grad(a2, d3)
        d2 = conv3d(d3, flip_transpose(self.w[2]), None, mask=a2)     # through relu(a2)
        dw2, db2 = conv3d_weight_grad(a1, d2)
        d1 = conv3d(d2, flip_transpose(self.w[1]), None, mask=a1)     # through relu(a1)
        dw1, db1 = conv3d_weight_grad(x1, d1)
        return [dw1, dw2, dw3, db1, db2, db3]

    def adam(self, grads, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        L = oat.lib()
        for p, gr, m, v in zip(self.parameters(), grads, self.m, self.v):
            oat._check(L.oat_adam_step(_ptr(p), _ptr(gr), _ptr(m), _ptr(v), p.numel(), lr, b1, b2,
                                       eps, self.step, _stream()))


def _rms(t: torch.Tensor) -> float:
    return max(float(t.double().pow(2).mean()) ** 0.5, 1e-30)


@dataclass
class TrainLog:
    loss: List[float] = field(default_factory=list)


def training_pairs(plan, phantoms, mu_rel: float = 1e-3, eps: float = 1e-3, iters: int = 10,
                   noise: float = 0.01, seed: int = 0):
    """(input, target) pairs from `iters` plain PLS-TV iterations per phantom:
    input = -g_k / rms(g_k), target = (a_true - a_k) / rms(a_true - a_k), both
    BF16, for the iterates a_k of pls_tv on u = H a_true + noise."""
    pairs = []
    gen = torch.Generator(device="cuda").manual_seed(seed)
    for a_true in phantoms:
        a_true = a_true.float().cuda()
        clean = plan.project(a_true)
        u = clean + noise * float(clean.abs().max()) * torch.randn(clean.shape, device="cuda",
                                                                   generator=gen)
        mu = mu_rel * float(u.double().pow(2).sum()) / (a_true.numel() * eps)
        for a_k, g_k in recon.pls_tv_iterates(plan, u, mu=mu, eps=eps, iters=iters):
            e = a_true - a_k
            pairs.append(((-g_k / _rms(g_k)).to(torch.bfloat16), (e / _rms(e)).to(torch.bfloat16)))
    return pairs


def train(model: Preconditioner, pairs, epochs: int = 5, lr: float = 1e-3, seed: int = 0,
          log: Optional[TrainLog] = None) -> TrainLog:
    """Adam on the mean squared error between z(input) and target, one pair
    per step, pairs in a seeded random order each epoch."""
    log = log or TrainLog()
    g = torch.Generator().manual_seed(seed)
    for _ in range(epochs):
        for i in torch.randperm(len(pairs), generator=g).tolist():
            x, t = pairs[i]
            z = model.forward(x, keep=True)
            loss, dz = mse(z, t)
            model.adam(model.backward(dz), lr=lr)
            log.loss.append(loss)
    log.loss = [float(v) for v in log.loss]
    return log


def _direction(cands, s: torch.Tensor, angle: float):
    """The first candidate direction c (name, tensor) whose angle with the
    steepest-descent direction s = -g is small enough,
    <c, s> >= angle ||c|| ||s||, else s itself (a plain step).  Returns
    (name, direction, cosine)."""
    ss = recon._dot(s, s) ** 0.5
    for name, c in cands:
        cn = recon._dot(c, c) ** 0.5
        cos = recon._dot(c, s) / max(cn * ss, 1e-300)
        if cos >= angle:
            return name, c, cos
    return "plain", s, 1.0


def pls_tv_learned(plan, u: torch.Tensor, model: Preconditioner, mu: float, eps: float,
                   iters: int = 20, storage=torch.float32, target: Optional[float] = None,
                   observe: Optional[Callable[[int, torch.Tensor], None]] = None,
                   switch: float = 0.4, powell: float = 0.2):
    """PLS-TV with the learned direction: nonlinear CG on the same objective
    and with the same line search as recon.pls_tv.  Its direction is
    z + beta d, with z = the network applied to -g (scaled to unit RMS and
    back) and beta = max(0, <z, s - s_prev> / <z_prev, s_prev>) (s = -g);
    beta = 0 when successive gradients are far from orthogonal
    (|<s, s_prev>| >= powell ||s||^2, Powell's restart).  A direction whose
    cosine with -g is below `switch` is replaced by z alone; once z also
    falls below it, the run goes on as the plain iteration (recon.pls_tv's
    directions, beta of Polak-Ribiere, clipped at 0) to the end.  Stops after
    `iters` iterations or once ||u - H a|| / ||u|| <= target.
    `observe(k, a)` is called with every iterate; the recorded times leave
    out its calls.  Returns a recon.PLSResult whose `directions` give each
    step's direction ("cg", "learned" or "plain") and its cosine with -g."""
    t0 = time.perf_counter()
    u = u.float().contiguous()
    unorm = max(recon._dot(u, u) ** 0.5, 1e-300)

    def H(x):
        return plan.project(x.to(storage).contiguous(), out_dtype=storage).float()

    def HT(y):
        return plan.backproject(y.to(storage).contiguous(), out_dtype=storage).float()

    def net(v):
        sc = _rms(v)
        return model.forward(v / sc).float() * sc

    a = torch.zeros(plan.image_shape, device=u.device, dtype=torch.float32)
    r = u.clone()
    tv, tg, w = recon.tv_eps(a, eps)
    g = -2.0 * HT(r) + mu * tg
    s = -g
    z = net(s)
    kind, d, cos = _direction([("learned", z)], s, switch)
    res = recon.PLSResult(a)
    res.residuals.append(1.0)
    res.objective.append(unorm ** 2 + mu * tv)
    res.times.append(time.perf_counter() - t0)
    if observe is not None:                           # not counted in the times
        t_obs = time.perf_counter()
        observe(0, a)
        t0 += time.perf_counter() - t_obs
    zs = recon._dot(z, s)
    for _ in range(iters):
        res.directions.append((kind, cos))
        Hd = H(d)
        dx, dy, dz = recon.forward_diff(d)
        curv = float((w.double() * (dx * dx + dy * dy + dz * dz).double()).sum())
        den = 2.0 * recon._dot(Hd, Hd) + mu * curv
        slope = recon._dot(g, d)
        if den <= 0.0 or slope >= 0.0:
            break
        t = -slope / den
        a = a + t * d
        r = r - t * Hd
        tv, tg, w = recon.tv_eps(a, eps)
        g = -2.0 * HT(r) + mu * tg
        s_new = -g
        ss_new = recon._dot(s_new, s_new)
        if kind == "plain":
            ss = recon._dot(s, s)
            beta = max(0.0, (ss_new - recon._dot(s_new, s)) / ss) if ss > 0 else 0.0
            d = s_new + beta * d
            if recon._dot(s_new, d) <= 0.0:
                d = s_new
            cos = recon._dot(d, s_new) / max((recon._dot(d, d) * ss_new) ** 0.5, 1e-300)
        else:
            z_new = net(s_new)
            restart = abs(recon._dot(s_new, s)) >= powell * ss_new
            beta = max(0.0, recon._dot(z_new, s_new - s) / zs) if zs > 0 and not restart else 0.0
            cands = [("cg", z_new + beta * d)] if beta > 0.0 else []
            kind, d, cos = _direction(cands + [("learned", z_new)], s_new, switch)
            zs = recon._dot(z_new, s_new)
        s = s_new
        rn = recon._dot(r, r)
        res.residuals.append(rn ** 0.5 / unorm)
        res.objective.append(rn + mu * tv)
        res.times.append(time.perf_counter() - t0)   # after FP64 dots: the device is synced
        if observe is not None:
            t_obs = time.perf_counter()
            observe(len(res.residuals) - 1, a)
            t0 += time.perf_counter() - t_obs
        if target is not None and res.residuals[-1] <= target:
            break
    res.image = a
    return res
