"""The learned preconditioner's kernels (include/oat_cnn.h) against plain
PyTorch FP64 CPU references, and its use inside PLS-TV.

CPU: argument checks of the C ABI; the adjoint convolution's weights.
GPU: every convolution shape with ReLU and masks, FP32 and BF16 activations;
weight/bias gradients; Adam; the loss; whole-model gradients; a short
training run; the learned PLS-TV iteration.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_1304_2017_amd import oat, precond, recon, synth


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ref_conv(x, w, b=None):
    """x [C_in, D, H, W], w [C_out, C_in, 27] -> 'same' convolution in FP64 on the CPU."""
    co, ci, _ = w.shape
    y = F.conv3d(x.double()[None].cpu(), w.double().cpu().reshape(co, ci, 3, 3, 3),
                 None if b is None else b.double().cpu(), padding=1)
    return y[0]


def _rel(a, b):
    a = a.detach().double().cpu().reshape(-1)
    b = b.detach().double().cpu().reshape(-1)
    return float((a - b).norm() / b.norm())


def test_cnn_abi_rejects_bad_arguments():
    L = oat.lib()
    vp = ctypes.c_void_p
    dummy = vp(16)
    assert L.oat_conv3d_forward(None, 0, 1, 4, 4, 4, dummy, None, 16, dummy, 0, 0, None, None) \
        == oat.OAT_ERR_ARG
    assert L.oat_conv3d_forward(dummy, 0, 3, 4, 4, 4, dummy, None, 16, vp(32), 0, 0, None, None) \
        == oat.OAT_ERR_ARG
    assert L.oat_conv3d_forward(dummy, 7, 1, 4, 4, 4, dummy, None, 16, vp(32), 0, 0, None, None) \
        == oat.OAT_ERR_DTYPE
    assert L.oat_conv3d_forward(dummy, 0, 1, 0, 4, 4, dummy, None, 16, vp(32), 0, 0, None, None) \
        == oat.OAT_ERR_ARG
    assert L.oat_conv3d_backward_weight_workspace(3, 16, 4, 4, 4) == 0
    need = L.oat_conv3d_backward_weight_workspace(16, 16, 9, 9, 9)
    assert need == 4 * (8 + 1) * (16 * 16 * 27 + 16)     # 2^3 tiles and one group of them
    assert L.oat_conv3d_backward_weight(dummy, 0, dummy, 0, 16, 16, 9, 9, 9, dummy, None, dummy,
                                        need - 1, None) == oat.OAT_ERR_ARG
    assert L.oat_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None) \
        == oat.OAT_ERR_ARG
    assert L.oat_mse(dummy, 0, dummy, 0, 0, dummy, dummy, dummy, None) == oat.OAT_ERR_ARG
    assert "bad argument" in oat.last_error()


def test_adjoint_weights_give_the_transposed_convolution():
    g = torch.Generator().manual_seed(0)
    w = torch.randn((16, 1, 27), generator=g, dtype=torch.float64)
    x = torch.randn((1, 6, 5, 7), generator=g, dtype=torch.float64)
    y = torch.randn((16, 6, 5, 7), generator=g, dtype=torch.float64)
    lhs = float((_ref_conv(x, w) * y).sum())
    rhs = float((x * _ref_conv(y, precond.flip_transpose(w))).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


class _DenseCG:
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


class _MapModel:
    """Stands in for the network: z = f(x)."""

    def __init__(self, f):
        self.f = f

    def forward(self, x):
        return self.f(x)


def _dense_problem():
    shape = (4, 5, 6)
    plan = _DenseCG(shape, 150, 11)
    g = torch.Generator().manual_seed(12)
    truth = torch.zeros(shape, dtype=torch.float64)
    truth[1:3, 1:4, 2:5] = 1.0
    u = plan.A @ truth.reshape(-1) + 0.01 * torch.randn(150, generator=g, dtype=torch.float64)
    return plan, u.reshape(150, 1).float()


def test_learned_iteration_with_switch_above_one_is_the_plain_iteration():
    """No direction has a cosine above 1 with -g, so every step is the plain
    one: the iterates are recon.pls_tv's, bit for bit."""
    plan, u = _dense_problem()
    model = _MapModel(lambda x: torch.flip(x, dims=[0]))
    plain = recon.pls_tv(plan, u, mu=0.05, eps=0.1, iters=15)
    res = precond.pls_tv_learned(plan, u, model, mu=0.05, eps=0.1, iters=15, switch=1.5)
    assert res.residuals == plain.residuals and res.objective == plain.objective
    assert torch.equal(res.image, plain.image)
    assert {k for k, _ in res.directions} == {"plain"}


def test_learned_iteration_with_the_identity_network_is_polak_ribiere_cg():
    """z = -g makes the learned beta <z, s - s_prev> / <z_prev, s_prev> the
    Polak-Ribiere beta of the plain iteration; with no restarts and any
    descent direction accepted the two runs agree to rounding."""
    plan, u = _dense_problem()
    model = _MapModel(lambda x: x.clone())
    plain = recon.pls_tv(plan, u, mu=0.05, eps=0.1, iters=15)
    res = precond.pls_tv_learned(plan, u, model, mu=0.05, eps=0.1, iters=15, switch=1e-12,
                                 powell=1e30)
    assert len(res.objective) == len(plain.objective)
    np.testing.assert_allclose(res.objective, plain.objective, rtol=1e-5)
    assert _rel(res.image, plain.image) < 1e-4


def test_learned_iteration_switches_to_plain_for_good():
    """A network whose output drifts away from -g: the learned and CG steps
    all keep a cosine of at least `switch` with -g, the first step below it
    turns the run into the plain iteration to the end, and the objective
    never rises."""
    plan, u = _dense_problem()
    g = torch.Generator().manual_seed(13)
    fixed = torch.randn(plan.image_shape, generator=g)
    fixed = fixed / fixed.pow(2).mean().sqrt()
    model = _MapModel(lambda x: 0.3 * x + fixed)
    res = precond.pls_tv_learned(plan, u, model, mu=0.05, eps=0.1, iters=20, switch=0.3)
    kinds = [k for k, _ in res.directions]
    assert "plain" in kinds and kinds[0] != "plain"
    first = kinds.index("plain")
    assert all(k == "plain" for k in kinds[first:])
    assert all(c >= 0.3 for k, c in res.directions[:first])
    obj = res.objective
    assert all(obj[i + 1] <= obj[i] * (1 + 1e-6) for i in range(len(obj) - 1))


def test_direction_takes_the_first_candidate_close_enough_to_steepest_descent():
    s = torch.tensor([1.0, 0.0, 0.0])
    far, near = torch.tensor([0.1, 1.0, 0.0]), torch.tensor([1.0, 1.0, 0.0])
    name, d, cos = precond._direction([("cg", far), ("learned", near)], s, 0.5)
    assert name == "learned" and torch.equal(d, near) and cos == pytest.approx(2 ** -0.5)
    name, d, cos = precond._direction([("cg", far)], s, 0.5)
    assert name == "plain" and torch.equal(d, s) and cos == 1.0


gpu = pytest.mark.gpu


@gpu
@pytest.mark.parametrize("ci,co", [(1, 16), (16, 16), (16, 1), (1, 1)])
@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("shape", [(13, 11, 9), (5, 7, 70)])
def test_conv3d_forward_matches_reference(ci, co, dt, shape):
    """Every layer shape against a PyTorch FP64 convolution; (5, 7, 70) spans
    several tiles along x (64 or 32 voxels wide) with ragged ends on all axes."""
    _say(f"[gpu] conv3d {ci}->{co} {dt} {shape}")
    g = torch.Generator().manual_seed(ci * 100 + co)
    x = torch.randn((ci,) + shape, generator=g).to(dt)
    w = torch.randn((co, ci, 27), generator=g) * 0.2
    b = torch.randn((co,), generator=g)
    y = precond.conv3d(x.cuda(), w.cuda(), b.cuda())
    ref = _ref_conv(x.float(), w, b)
    e = _rel(y, ref)
    tol = 1e-6 if dt == torch.float32 else 8e-3
    _say(f"  rel {e:.3e}")
    assert e < tol
    # ReLU, then an output mask
    yr = precond.conv3d(x.cuda(), w.cuda(), b.cuda(), relu=True)
    assert _rel(yr, ref.clamp(min=0)) < tol
    m = torch.randn((co,) + shape, generator=g).to(dt)
    ym = precond.conv3d(x.cuda(), w.cuda(), b.cuda(), mask=m.cuda())
    assert _rel(ym, ref * (m.double() > 0)) < tol


@gpu
@pytest.mark.parametrize("ci,co", [(1, 16), (16, 16), (16, 1)])
def test_conv3d_weight_grad_matches_autograd(ci, co):
    g = torch.Generator().manual_seed(7 + ci + co)
    x = torch.randn((ci, 17, 9, 10), generator=g)
    dy = torch.randn((co, 17, 9, 10), generator=g)
    dw, db = precond.conv3d_weight_grad(x.cuda(), dy.cuda())
    w = torch.zeros((co, ci, 3, 3, 3), dtype=torch.float64, requires_grad=True)
    b = torch.zeros((co,), dtype=torch.float64, requires_grad=True)
    y = F.conv3d(x.double()[None], w, b, padding=1)[0]
    (y * dy.double()).sum().backward()
    ew, eb = _rel(dw, w.grad.reshape(co, ci, 27)), _rel(db, b.grad)
    _say(f"[gpu] conv3d weight grad {ci}->{co}: rel {ew:.3e} bias {eb:.3e}")
    assert ew < 1e-5 and eb < 1e-5
    # deterministic: the same call twice
    dw2, db2 = precond.conv3d_weight_grad(x.cuda(), dy.cuda())
    assert torch.equal(dw, dw2) and torch.equal(db, db2)


@gpu
@pytest.mark.parametrize("shape", [(13, 11, 9), (19, 17, 21), (8, 8, 8)])
def test_bf16_16ch_layers_on_matrix_cores(shape):
    """BF16 16 -> 16 layers run on the matrix cores (BF16 operands, weights
    rounded to BF16, FP32 accumulation).  Against FP64 on the same rounded
    weights and inputs only FP32 accumulation remains (FP32 output) or the
    output's BF16 rounding (BF16 output); the weight gradient of BF16 x and
    dy is exact products summed in FP32."""
    g = torch.Generator().manual_seed(sum(shape))
    x = torch.randn((16,) + shape, generator=g).to(torch.bfloat16)
    w = torch.randn((16, 16, 27), generator=g) * 0.2
    b = torch.randn((16,), generator=g)
    wb = w.to(torch.bfloat16).float()
    ref = _ref_conv(x.float(), wb, b)
    y32 = precond.conv3d(x.cuda(), w.cuda(), b.cuda(), out_dtype=torch.float32)
    y16 = precond.conv3d(x.cuda(), w.cuda(), b.cuda())
    m = torch.randn((16,) + shape, generator=g).to(torch.bfloat16)
    ym = precond.conv3d(x.cuda(), w.cuda(), b.cuda(), relu=True, mask=m.cuda())
    e32, e16 = _rel(y32, ref), _rel(y16, ref)
    em = _rel(ym, ref.clamp(min=0) * (m.double() > 0))
    # element-wise: every output within its BF16 half-ulp (plus FP32 sums)
    d16 = (y16.double().cpu() - ref).abs() / ref.abs().clamp(min=1e-3)
    dy = torch.randn((16,) + shape, generator=g).to(torch.bfloat16)
    dw, db = precond.conv3d_weight_grad(x.cuda(), dy.cuda())
    wr = torch.zeros((16, 16, 3, 3, 3), dtype=torch.float64, requires_grad=True)
    br = torch.zeros((16,), dtype=torch.float64, requires_grad=True)
    (F.conv3d(x.double()[None], wr, br, padding=1)[0] * dy.double()).sum().backward()
    ew, eb = _rel(dw, wr.grad.reshape(16, 16, 27)), _rel(db, br.grad)
    _say(f"[gpu] MFMA 16->16 {shape}: fwd FP32-out rel {e32:.3e}, BF16-out rel {e16:.3e} "
         f"(max {float(d16.max()):.2e}), relu+mask {em:.3e}; dW rel {ew:.3e}, db rel {eb:.3e}")
    assert e32 < 1e-5 and e16 < 2.5e-3 and em < 2.5e-3
    assert float(d16.max()) < 2 ** -8 + 1e-4
    assert ew < 1e-5 and eb < 1e-5
    dw2, db2 = precond.conv3d_weight_grad(x.cuda(), dy.cuda())
    assert torch.equal(dw, dw2) and torch.equal(db, db2)


@gpu
def test_adam_and_mse_match_their_formulas():
    g = torch.Generator().manual_seed(3)
    p = torch.randn(1000, generator=g)
    m = torch.zeros(1000)
    v = torch.zeros(1000)
    pd, md, vd = p.cuda(), m.cuda(), v.cuda()
    P, M, V = p.double(), m.double(), v.double()
    L = oat.lib()
    for step in range(1, 4):
        gr = torch.randn(1000, generator=g)
        oat._check(L.oat_adam_step(precond._ptr(pd), precond._ptr(gr.cuda()), precond._ptr(md),
                                   precond._ptr(vd), 1000, 1e-2, 0.9, 0.999, 1e-8, step,
                                   precond._stream()))
        G = gr.double()
        M = 0.9 * M + 0.1 * G
        V = 0.999 * V + 0.001 * G * G
        P = P - 1e-2 * (M / (1 - 0.9 ** step)) / ((V / (1 - 0.999 ** step)).sqrt() + 1e-8)
    assert _rel(pd, P) < 1e-6
    y = torch.randn((3, 5, 7), generator=g)
    t = torch.randn((3, 5, 7), generator=g)
    loss, dy = precond.mse(y.cuda(), t.cuda())
    torch.cuda.synchronize()
    want = float(((y.double() - t.double()) ** 2).mean())
    assert abs(float(loss) - want) < 1e-6 * want
    assert _rel(dy, 2 * (y.double() - t.double()) / y.numel()) < 1e-6


@gpu
def test_model_gradient_matches_autograd():
    _say("[gpu] preconditioner gradient")
    model = precond.Preconditioner(seed=1, storage=torch.float32, init_scale=1.0)
    g = torch.Generator().manual_seed(5)
    x = torch.randn((12, 10, 9), generator=g)
    t = torch.randn((12, 10, 9), generator=g)
    z = model.forward(x.cuda(), keep=True)
    loss, dz = precond.mse(z, t.cuda())
    grads = model.backward(dz)
    W = [w.double().cpu().reshape(w.shape[0], w.shape[1], 3, 3, 3).requires_grad_(True) for w in model.w]
    B = [b.double().cpu().requires_grad_(True) for b in model.b]
    a = x.double()[None, None]
    a1 = F.relu(F.conv3d(a, W[0], B[0], padding=1))
    a2 = F.relu(F.conv3d(a1, W[1], B[1], padding=1))
    zr = (a + F.conv3d(a2, W[2], B[2], padding=1))[0, 0]
    assert _rel(z, zr) < 1e-5
    lr = ((zr - t.double()) ** 2).mean()
    lr.backward()
    assert abs(float(loss) - float(lr)) < 1e-5 * float(lr)
    for gk, ref in zip(grads, [w.grad for w in W] + [b.grad for b in B]):
        e = _rel(gk, ref.reshape(gk.shape))
        assert e < 1e-4, e


@gpu
def test_training_lowers_the_loss():
    """Learn a fixed 3-D smoothing of the input: the loss must fall well below
    its starting value."""
    _say("[gpu] preconditioner training")
    g = torch.Generator().manual_seed(9)
    ker = torch.tensor([0.25, 0.5, 0.25], dtype=torch.float64)
    k3 = (ker[:, None, None] * ker[None, :, None] * ker[None, None, :]).reshape(1, 1, 27)
    pairs = []
    for _ in range(8):
        x = torch.randn((16, 16, 16), generator=g)
        t = _ref_conv(x[None], k3)[0].float()
        pairs.append((x.to(torch.bfloat16).cuda(), t.to(torch.bfloat16).cuda()))
    model = precond.Preconditioner(seed=2)
    log = precond.train(model, pairs, epochs=40, lr=3e-3)
    first, last = np.mean(log.loss[:8]), np.mean(log.loss[-8:])
    _say(f"  loss {first:.4f} -> {last:.4f}")
    assert last < 0.3 * first


@gpu
def test_learned_pls_tv_descends():
    """With any network the learned iteration keeps the objective decreasing
    (directions far from -g hand the run to the plain iteration)."""
    from paper_1304_2017_amd.oat import Plan
    _say("[gpu] learned PLS-TV")
    geom, balls, _ = synth.config_small(2)
    plan = Plan(geom.with_detectors(np.arange(0, 64, 2)), 0)
    u = torch.from_numpy(synth.nwave_balls(plan.geom, balls)).float().cuda()
    model = precond.Preconditioner(seed=3, init_scale=1.0)
    res = precond.pls_tv_learned(plan, u, model, mu=2e-3, eps=1e-2, iters=8)
    obj = res.objective
    _say(f"  residuals {['%.4f' % v for v in res.residuals]}")
    assert all(obj[i + 1] <= obj[i] * (1 + 1e-4) for i in range(len(obj) - 1))
    assert res.residuals[-1] < res.residuals[0]
