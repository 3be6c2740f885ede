"""Autograd wrappers and the PLS (Sec. IV.A-B) reconstruction.

CPU: the smoothness penalty's normal operator is checked against its
definition by exact identities.  GPU: the autograd gradient is checked by
finite differences and against the adjoint; the CG iterates are compared
with the same recursion run on the FP64 oracle's operators.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1304_2017_amd import recon, synth


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_smoothness_normal_is_half_gradient_of_penalty():
    g = torch.Generator().manual_seed(0)
    a = torch.randn((5, 6, 7), generator=g, dtype=torch.float64)
    b = torch.randn((5, 6, 7), generator=g, dtype=torch.float64)
    # <L^T L a, b> = <L a, L b>: polarisation of R
    lab = 0.25 * (float(recon.smoothness_penalty(a + b)) - float(recon.smoothness_penalty(a - b)))
    assert abs(float((recon.smoothness_normal(a) * b).sum()) - lab) < 1e-10 * abs(lab)
    # R(a) = <L^T L a, a>
    assert abs(float((recon.smoothness_normal(a) * a).sum()) -
               float(recon.smoothness_penalty(a))) < 1e-10 * float(recon.smoothness_penalty(a))
    # brute-force definition of R on a tiny grid
    t = torch.arange(8, dtype=torch.float64).reshape(2, 2, 2) ** 2
    want = 0.0
    for z in range(2):
        for y in range(2):
            for x in range(2):
                if z: want += float(t[z, y, x] - t[z - 1, y, x]) ** 2
                if y: want += float(t[z, y, x] - t[z, y - 1, x]) ** 2
                if x: want += float(t[z, y, x] - t[z, y, x - 1]) ** 2
    assert float(recon.smoothness_penalty(t)) == want


def _small_geom(Q=32):
    n, dx = 16, 0.5
    o = synth.centred_origin(n, dx)
    return synth.Geometry(n, n, n, dx, o, o, o, synth.fibonacci_sphere(Q, 15.0), 200, 0.1,
                          0.0, 1.5, 1.0)


@pytest.mark.gpu
def test_autograd_gradient_finite_differences():
    from paper_1304_2017_amd.oat import Plan
    _say("[gpu] autograd FD 16^3")
    geom = _small_geom()
    plan = Plan(geom, 0)
    dev = torch.device("cuda", 0)
    g = torch.Generator().manual_seed(1)
    x0 = torch.rand(geom.shape, generator=g).to(dev)
    y = torch.randn(plan.data_shape, generator=g).to(dev)
    v = torch.randn(geom.shape, generator=g).to(dev)
    x = x0.clone().requires_grad_(True)
    loss = 0.5 * ((recon.project(x, plan) - y) ** 2).sum()
    loss.backward()
    grad = x.grad.detach()
    # the backward pass is exactly the adjoint kernel
    direct = plan.backproject((plan.project(x0) - y).contiguous())
    assert torch.allclose(grad, direct, rtol=1e-6, atol=1e-6 * float(direct.abs().max()))

    def L(t):
        return 0.5 * float((plan.project(t).double() - y.double()).pow(2).sum())
    eps = 1e-2
    fd = (L(x0 + eps * v) - L(x0 - eps * v)) / (2 * eps)
    an = float((grad.double() * v.double()).sum())
    _say(f"  directional derivative FD {fd:.6e} analytic {an:.6e}")
    assert abs(fd - an) <= 2e-3 * abs(an)
    # gradient of the adjoint wrapper is the projector
    d = y.clone().requires_grad_(True)
    out = (recon.backproject(d, plan) * x0).sum()
    out.backward()
    assert torch.allclose(d.grad, plan.project(x0), rtol=1e-6,
                          atol=1e-6 * float(d.grad.abs().max()))


@pytest.mark.gpu
@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_pls_cg_matches_oracle_recursion(mu):
    from oracle import ref
    from paper_1304_2017_amd.oat import Plan
    _say(f"[gpu] PLS CG mu={mu}")
    geom, balls, _ = synth.config_small(0)
    geom = geom.with_detectors(np.arange(0, 64, 2))
    plan = Plan(geom, 0)
    u = synth.nwave_balls(geom, balls).astype(np.float32).astype(np.float64)
    iters = 5
    res = recon.pls_cg(plan, torch.from_numpy(u).float().cuda(), mu=mu, iters=iters)
    gd = geom.as_dict()

    def A(p):
        out = ref.backproject(gd, ref.project(gd, p))
        if mu:
            out = out + mu * recon.smoothness_normal(torch.from_numpy(p)).numpy()
        return out
    a = np.zeros(geom.shape)
    r = ref.backproject(gd, u)
    p = r.copy()
    rr = float(np.vdot(r, r))
    for _ in range(iters):
        Ap = A(p)
        alpha = rr / float(np.vdot(p, Ap))
        a = a + alpha * p
        r = r - alpha * Ap
        rn = float(np.vdot(r, r))
        p = r + (rn / rr) * p
        rr = rn
    got = res.image.double().cpu().numpy()
    e = float(np.linalg.norm(got - a) / np.linalg.norm(a))
    _say(f"  iterate rel {e:.3e}; residuals {['%.4f' % v for v in res.residuals]}")
    assert e < 1e-3
    # CG minimises the objective monotonically along its Krylov space
    obj = res.objective
    assert all(obj[i + 1] <= obj[i] * (1 + 1e-6) for i in range(len(obj) - 1))
    assert res.residuals[-1] < res.residuals[0]
