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

    def LtL(p):
        # L^T L of the penalty R(a) = sum over axes of (a_n - a_{n - axis})^2,
        # written out here in numpy
        out = np.zeros_like(p)
        for ax in range(3):
            d = np.diff(p, axis=ax)
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[ax] = slice(1, None)
            lo[ax] = slice(None, -1)
            out[tuple(hi)] += d
            out[tuple(lo)] -= d
        return out

    def A(p):
        out = ref.backproject(gd, ref.project(gd, p))
        if mu:
            out = out + mu * LtL(p)
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
    # about 10x the measured FP32 error of five iterations
    assert e < 2e-6
    # CG minimises the objective monotonically along its Krylov space
    obj = res.objective
    assert all(obj[i + 1] <= obj[i] * (1 + 1e-6) for i in range(len(obj) - 1))
    assert res.residuals[-1] < res.residuals[0]


# ---------------------------------------------------------------------------
# PLS with the smoothed total-variation penalty
# ---------------------------------------------------------------------------
def test_forward_diff_values_and_adjoint():
    g = torch.Generator().manual_seed(3)
    a = torch.randn((4, 5, 6), generator=g, dtype=torch.float64)
    gx, gy, gz = recon.forward_diff(a)
    # brute-force definition at a few nodes
    assert float(gx[1, 2, 3]) == float(a[1, 2, 4] - a[1, 2, 3])
    assert float(gy[3, 1, 0]) == float(a[3, 2, 0] - a[3, 1, 0])
    assert float(gz[2, 4, 5]) == float(a[3, 4, 5] - a[2, 4, 5])
    assert float(gx[0, 0, 5]) == 0.0 and float(gy[0, 4, 0]) == 0.0 and float(gz[3, 0, 0]) == 0.0
    # <D a, (p, q, r)> = <a, D^T (p, q, r)>
    p, q, r = (torch.randn((4, 5, 6), generator=g, dtype=torch.float64) for _ in range(3))
    lhs = float((gx * p).sum() + (gy * q).sum() + (gz * r).sum())
    rhs = float((a * recon.forward_diff_adj(p, q, r)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_tv_closed_forms_and_gradient():
    eps = 0.05
    c = torch.full((3, 4, 5), 2.0, dtype=torch.float64)
    tv, grad, _ = recon.tv_eps(c, eps)
    assert abs(tv - 60 * eps) < 1e-12 and float(grad.abs().max()) == 0.0
    # ramp along x with slope s: |grad| = s except in the last x slice
    s = 0.3
    ramp = s * torch.arange(5, dtype=torch.float64)[None, None, :].expand(3, 4, 5).contiguous()
    tv, _, _ = recon.tv_eps(ramp, eps)
    want = 3 * 4 * (4 * np.sqrt(s * s + eps * eps) + eps)
    assert abs(tv - want) < 1e-12 * want
    # gradient against central differences
    g = torch.Generator().manual_seed(4)
    a = torch.randn((4, 4, 4), generator=g, dtype=torch.float64)
    v = torch.randn((4, 4, 4), generator=g, dtype=torch.float64)
    _, grad, _ = recon.tv_eps(a, eps)
    h = 1e-6
    fd = (recon.tv_eps(a + h * v, eps)[0] - recon.tv_eps(a - h * v, eps)[0]) / (2 * h)
    an = float((grad * v).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)


class _DensePlan:
    """A dense random H on the CPU with the Plan interface (solver tests)."""

    def __init__(self, shape, m, seed):
        g = torch.Generator().manual_seed(seed)
        self.image_shape = shape
        self.data_shape = (m, 1)
        self.A = torch.randn((m, int(np.prod(shape))), generator=g, dtype=torch.float64) / m ** 0.5

    def project(self, x, out_dtype=None):
        return (self.A @ x.double().reshape(-1)).reshape(self.data_shape).to(x.dtype)

    def backproject(self, y, out_dtype=None):
        return (self.A.T @ y.double().reshape(-1)).reshape(self.image_shape).to(y.dtype)


def test_pls_tv_descends_to_the_minimiser():
    from scipy.optimize import minimize
    shape, mu, eps = (4, 5, 6), 0.05, 0.1
    plan = _DensePlan(shape, 150, 5)
    g = torch.Generator().manual_seed(6)
    truth = torch.zeros(shape, dtype=torch.float64)
    truth[1:3, 1:4, 2:5] = 1.0
    u = (plan.A @ truth.reshape(-1) + 0.01 * torch.randn(150, generator=g, dtype=torch.float64))
    u = u.reshape(150, 1)

    def F(x):
        t = torch.from_numpy(x).reshape(shape)
        r = u.reshape(-1) - plan.A @ t.reshape(-1)
        tv, grad, _ = recon.tv_eps(t, eps)
        return float(r @ r) + mu * tv, (-2 * plan.A.T @ r + mu * grad.reshape(-1)).numpy()

    opt = minimize(F, np.zeros(np.prod(shape)), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=5000, gtol=1e-12, ftol=1e-15))
    res = recon.pls_tv(plan, u.float(), mu=mu, eps=eps, iters=300)
    obj = res.objective
    assert all(obj[i + 1] <= obj[i] * (1 + 1e-5) for i in range(len(obj) - 1))
    got, _ = F(res.image.double().numpy().ravel())
    assert got - opt.fun <= 1e-4 * opt.fun


def test_checkpoint_resume_takes_the_same_steps(tmp_path):
    """A run continued from a checkpoint takes exactly the steps of an
    uninterrupted one (image, residuals and objective equal), for linear CG
    and for PLS-TV; the state file is plain data (weights-only load)."""
    shape = (4, 5, 6)
    plan = _DensePlan(shape, 150, 5)
    g = torch.Generator().manual_seed(7)
    u = (plan.A @ torch.rand(int(np.prod(shape)), generator=g, dtype=torch.float64)).reshape(150, 1)
    u = u.float()
    ck = str(tmp_path / "cg.pt")
    full = recon.pls_cg(plan, u, mu=0.05, iters=9)
    part = recon.pls_cg(plan, u, mu=0.05, iters=6, checkpoint=ck, every=3)
    st = torch.load(ck, weights_only=True)
    assert st["k"] == 6 and torch.equal(st["a"], part.image)
    cont = recon.pls_cg(plan, u, mu=0.05, iters=9, resume=ck)
    assert torch.equal(cont.image, full.image)
    assert cont.residuals == full.residuals and cont.objective == full.objective
    ck2 = str(tmp_path / "tv.pt")
    seen = []
    full = recon.pls_tv(plan, u, mu=0.05, eps=0.1, iters=12,
                        observe=lambda k, a: seen.append((k, a.clone())))
    assert [k for k, _ in seen] == list(range(13)) and torch.equal(seen[-1][1], full.image)
    assert not seen[0][1].any()                       # the start a = 0
    recon.pls_tv(plan, u, mu=0.05, eps=0.1, iters=8, checkpoint=ck2, every=4)
    assert torch.load(ck2, weights_only=True)["k"] == 8
    cont = recon.pls_tv(plan, u, mu=0.05, eps=0.1, iters=12, resume=ck2)
    assert torch.equal(cont.image, full.image)
    assert cont.residuals == full.residuals and cont.objective == full.objective
    assert len(cont.times) == len(full.times) == 13


def test_rmse_is_the_papers_definition():
    a = torch.tensor([[1.0, 2.0], [3.0, 5.0]])
    b = np.array([[1.0, 0.0], [3.0, 1.0]])
    assert recon.rmse(a, b) == pytest.approx(((4.0 + 16.0) / 4.0) ** 0.5, rel=1e-15)


@pytest.mark.gpu
def test_fbp_rmse_single_precision_matches_the_oracle():
    """Sec. V.B: single-precision FBP changes the RMSE against the phantom
    negligibly.  FP32 FBP of the analytic N-wave of the 32^3 balls against
    the FP64 oracle's, both measured against the balls' node samples."""
    from oracle import ref
    from paper_1304_2017_amd.oat import Plan
    geom, balls, phantom = synth.config_small(0)
    plan = Plan(geom, 0)
    u = synth.nwave_balls(geom, balls).astype(np.float32)
    f = plan.fbp(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    f_ref = ref.fbp(geom.as_dict(), u.astype(np.float64))
    e_gpu = recon.rmse(f.cpu(), phantom)
    e_ref = float(np.sqrt(np.mean((f_ref - phantom) ** 2)))
    _say(f"[gpu] FBP RMSE vs phantom: FP32 {e_gpu:.6e}, FP64 oracle {e_ref:.6e}")
    assert abs(e_gpu - e_ref) <= 1e-4 * e_ref


def _np_tv(a, eps):
    """Independent numpy form of TV_eps and its gradient (forward differences
    with zero across the far faces)."""
    d = [np.zeros_like(a) for _ in range(3)]
    d[0][:, :, :-1] = a[:, :, 1:] - a[:, :, :-1]
    d[1][:, :-1, :] = a[:, 1:, :] - a[:, :-1, :]
    d[2][:-1, :, :] = a[1:, :, :] - a[:-1, :, :]
    s = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + eps * eps)
    q = [di / s for di in d]
    grad = np.zeros_like(a)
    grad[:, :, 1:] += q[0][:, :, :-1]
    grad[:, :, :-1] -= q[0][:, :, :-1]
    grad[:, 1:, :] += q[1][:, :-1, :]
    grad[:, :-1, :] -= q[1][:, :-1, :]
    grad[1:, :, :] += q[2][:-1, :, :]
    grad[:-1, :, :] -= q[2][:-1, :, :]
    return s.sum(), grad, 1.0 / s


@pytest.mark.gpu
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_pls_tv_matches_oracle_recursion(storage):
    from oracle import ref
    from paper_1304_2017_amd.oat import Plan
    _say(f"[gpu] PLS-TV {storage}")
    geom, balls, _ = synth.config_small(1)
    geom = geom.with_detectors(np.arange(0, 64, 2))
    plan = Plan(geom, 0)
    u = synth.nwave_balls(geom, balls).astype(np.float32).astype(np.float64)
    mu, eps, iters = 2e-3, 1e-2, 5
    dt = torch.float32 if storage == "f32" else torch.bfloat16
    res = recon.pls_tv(plan, torch.from_numpy(u).float().cuda(), mu=mu, eps=eps, iters=iters,
                       storage=dt)
    gd = geom.as_dict()
    H = lambda x: ref.project(gd, x)
    HT = lambda y: ref.backproject(gd, y)
    a = np.zeros(geom.shape)
    r = u.copy()
    tv, tg, w = _np_tv(a, eps)
    g = -2 * HT(r) + mu * tg
    d = -g
    for _ in range(iters):
        Hd = H(d)
        dd = [np.zeros_like(d) for _ in range(3)]
        dd[0][:, :, :-1] = np.diff(d, axis=2)
        dd[1][:, :-1, :] = np.diff(d, axis=1)
        dd[2][:-1, :, :] = np.diff(d, axis=0)
        t = -np.vdot(g, d) / (2 * np.vdot(Hd, Hd) + mu * np.sum(w * (dd[0] ** 2 + dd[1] ** 2 + dd[2] ** 2)))
        a = a + t * d
        r = r - t * Hd
        tv, tg, w = _np_tv(a, eps)
        gn = -2 * HT(r) + mu * tg
        beta = max(0.0, np.vdot(gn, gn - g) / np.vdot(g, g))
        d = -gn + beta * d
        if np.vdot(gn, d) >= 0:
            d = -gn
        g = gn
    got = res.image.double().cpu().numpy()
    e = float(np.linalg.norm(got - a) / np.linalg.norm(a))
    _say(f"  iterate rel {e:.3e}; residuals {['%.4f' % v for v in res.residuals]}")
    # about 10x the measured errors (1.5e-7 FP32; 6e-4 with BF16 storage of
    # the operator inputs and outputs)
    assert e < (2e-6 if storage == "f32" else 6e-3)
    obj = res.objective
    assert all(obj[i + 1] <= obj[i] * (1 + 1e-4) for i in range(len(obj) - 1))
