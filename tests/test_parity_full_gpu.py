"""Parity at the full benchmark size (256^3 nodes at 0.1 mm, 2048 transducers,
1024 samples), in the launch configuration bench.py times, on outputs the
FP64 oracle can compute one by one:

- H and G: whole rows of a few transducers (the oracle evaluates rows);
- H^T: the full image for data that is nonzero on a few transducers (the
  kernel still walks every transducer's points), among them one transducer
  in each of G^T's 16 windows of 128, so every window's fixed-point scale,
  the FP64 sums of all windows and every slice of a brick's windows carry
  data;
- the adjoint identity <Hx, y> = <x, H^T y> with random x and y on every
  transducer;
- FBP: sampled voxels of the full image for seeded Gaussian data.
Each comparison gates the relative L2 and max |error| / max |reference|.
"""
import sys

import numpy as np
import pytest

from checks import BF16_ELEM, check
from paper_1304_2017_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from oracle import ref  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def large():
    from paper_1304_2017_amd.oat import Plan
    _say("[gpu-full] building 256^3 workload")
    geom, _, img = synth.config_large(0, dtype=np.float32)
    plan = Plan(geom, 0)
    return geom, img, plan


def test_full_size_project_rows(large):
    geom, img, plan = large
    rows = np.array([0, 701, 1500, 2047], dtype=np.int32)
    _say(f"[gpu-full] H and G, oracle rows {rows.tolist()}")
    x = torch.from_numpy(img).cuda()
    p = plan.project(x)
    g = plan.project(x, srt_only=True)
    torch.cuda.synchronize()
    p = p.double().cpu().numpy()[rows]
    g = g.double().cpu().numpy()[rows]
    gd = geom.as_dict()
    img64 = img.astype(np.float64)
    check("G rows", g, ref.srt(gd, img64, rows=rows), 5e-7)
    check("H rows", p, ref.project(gd, img64, rows=rows), 1e-5)


def test_full_size_project_rows_bf16(large):
    geom, img, plan = large
    rows = np.array([333, 1777], dtype=np.int32)
    _say("[gpu-full] H BF16")
    xb = torch.from_numpy(img).to(torch.bfloat16).cuda()
    p = plan.project(xb, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    p = p.double().cpu().numpy()[rows]
    img_b = xb.double().cpu().numpy()
    check("H bf16 rows", p, ref.project(geom.as_dict(), img_b, rows=rows), 2e-3, BF16_ELEM)


def test_full_size_backproject_two_transducers(large):
    geom, img, plan = large
    rows = np.array([3, 1999], dtype=np.int32)
    _say(f"[gpu-full] H^T with data on transducers {rows.tolist()}")
    rng = np.random.default_rng(11)
    y = np.zeros((geom.n_det, geom.n_t), dtype=np.float32)
    y[rows] = rng.normal(size=(rows.size, geom.n_t)).astype(np.float32)
    a = plan.backproject(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    a = a.double().cpu().numpy()
    want = ref.backproject(geom.as_dict(), y[rows].astype(np.float64), rows=rows)
    check("H^T", a, want, 1e-5)


def window_rows(n_det, window=128):
    """One transducer in every window of `window`, at a position within the
    window that moves from window to window (first, last and in between)."""
    rows = []
    for w in range((n_det + window - 1) // window):
        size = min(window, n_det - w * window)
        rows.append(w * window + (w * 37) % size)
    return np.array(rows, dtype=np.int32)


def test_full_size_backproject_one_row_per_window(large):
    """Seeded data on one transducer in each of the 16 windows (and so in
    every brick slice), zero elsewhere: the whole H^T image against the
    oracle's sum over those rows."""
    geom, img, plan = large
    rows = window_rows(geom.n_det)
    assert rows.size == 16
    _say(f"[gpu-full] H^T with data on one transducer per window: {rows.tolist()}")
    rng = np.random.default_rng(14)
    y = np.zeros((geom.n_det, geom.n_t), dtype=np.float32)
    y[rows] = rng.normal(size=(rows.size, geom.n_t)).astype(np.float32)
    a = plan.backproject(torch.from_numpy(y).cuda())
    g = plan.backproject(torch.from_numpy(y).cuda(), srt_only=True)
    torch.cuda.synchronize()
    gd = geom.as_dict()
    y64 = y[rows].astype(np.float64)
    check("H^T 16 windows", a.double().cpu().numpy(), ref.backproject(gd, y64, rows=rows), 1e-5)
    check("G^T 16 windows", g.double().cpu().numpy(), ref.srt_adj(gd, y64, rows=rows), 1e-5)


def test_full_size_adjoint_identity(large):
    """<Hx, y> = <x, H^T y> at full size with seeded random x and y on all
    2048 transducers, every window and slice carrying data; bound
    1e-6 |Hx| |y| (both sides FP32 operators, inner products in FP64)."""
    geom, img, plan = large
    _say("[gpu-full] adjoint identity, random data on every transducer")
    gen = torch.Generator(device="cuda").manual_seed(15)
    x = torch.randn(geom.shape, device="cuda", generator=gen)
    y = torch.randn((geom.n_det, geom.n_t), device="cuda", generator=gen)
    Hx = plan.project(x)
    HTy = plan.backproject(y)
    torch.cuda.synchronize()
    lhs = float(torch.dot(Hx.double().ravel(), y.double().ravel()))
    rhs = float(torch.dot(x.double().ravel(), HTy.double().ravel()))
    scale = float(Hx.double().norm() * y.double().norm())
    _say(f"  <Hx,y> {lhs:.9e}  <x,H^T y> {rhs:.9e}  |diff| / (|Hx||y|) {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= 1e-6 * scale
    # and with the ellipsoid phantom as x
    xi = torch.from_numpy(img).cuda()
    Hxi = plan.project(xi)
    torch.cuda.synchronize()
    lhs = float(torch.dot(Hxi.double().ravel(), y.double().ravel()))
    rhs = float(torch.dot(xi.double().ravel(), HTy.double().ravel()))
    scale = float(Hxi.double().norm() * y.double().norm())
    _say(f"  phantom: |diff| / (|Hx||y|) {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_full_size_fbp_sampled_voxels(large):
    geom, img, plan = large
    _say("[gpu-full] FBP on sampled voxels")
    rng = np.random.default_rng(12)
    p = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32)
    f = plan.fbp(torch.from_numpy(p).cuda())
    torch.cuda.synchronize()
    f = f.double().cpu().numpy().ravel()
    vox = rng.choice(geom.n_vox, 3000, replace=False)
    want = ref.fbp(geom.as_dict(), p.astype(np.float64), voxels=vox)
    check("FBP voxels", f[vox], want, 1e-5)


def test_sphere_8192_shapes_on_64_transducers():
    """256^3 at 0.1 mm with every 128th of 8192 sphere transducers (45 mm):
    the whole H, H^T and FBP outputs against the oracle."""
    from paper_1304_2017_amd.oat import Plan
    geom_full, _, img = synth.config_e(0)
    geom = geom_full.with_detectors(np.arange(0, 8192, 128))
    _say(f"[gpu-full] 256^3 / 64 of 8192 sphere transducers")
    plan = Plan(geom, 0)
    gd = geom.as_dict()
    img64 = img.astype(np.float64)
    p = plan.project(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    p = p.double().cpu().numpy()
    check("H", p, ref.project(gd, img64), 1e-5)
    rng = np.random.default_rng(21)
    y = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32)
    a = plan.backproject(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    check("H^T", a.double().cpu().numpy(), ref.backproject(gd, y.astype(np.float64)), 1e-5)
    pf = p.astype(np.float32)
    f = plan.fbp(torch.from_numpy(pf).cuda())
    torch.cuda.synchronize()
    check("FBP", f.double().cpu().numpy(), ref.fbp(gd, pf.astype(np.float64)), 1e-5)


def test_paper_shape_rows_and_voxels():
    """210 x 210 x 440 at 0.14 mm, 64 x 90 ring views at 65 mm, t0 = 17.5 us:
    G and H rows and sampled FBP voxels against the oracle."""
    from paper_1304_2017_amd.oat import Plan
    geom, _, img = synth.config_p(0)
    _say("[gpu-full] paper shape 210x210x440 / 5760 ring views")
    plan = Plan(geom, 0)
    gd = geom.as_dict()
    img64 = img.astype(np.float64)
    rows = np.array([0, 1234, 2900, 5759], dtype=np.int32)
    x = torch.from_numpy(img).cuda()
    p = plan.project(x)
    g = plan.project(x, srt_only=True)
    torch.cuda.synchronize()
    check("G rows", g.double().cpu().numpy()[rows], ref.srt(gd, img64, rows=rows), 5e-7)
    check("H rows", p.double().cpu().numpy()[rows], ref.project(gd, img64, rows=rows), 1e-5)
    pn = p.float()
    f = plan.fbp(pn)
    torch.cuda.synchronize()
    vox = np.random.default_rng(22).choice(geom.n_vox, 2000, replace=False)
    check("FBP voxels", f.double().cpu().numpy().ravel()[vox],
          ref.fbp(gd, pn.double().cpu().numpy(), voxels=vox), 1e-5)


def test_full_size_bf16_backproject_and_fbp(large):
    """BF16 storage for H^T and FBP at full size (oracle fed the same
    BF16-rounded inputs); H^T repeats bit for bit."""
    geom, img, plan = large
    rows = np.array([17, 1024], dtype=np.int32)
    rng = np.random.default_rng(13)
    y = np.zeros((geom.n_det, geom.n_t), dtype=np.float32)
    y[rows] = rng.normal(size=(rows.size, geom.n_t)).astype(np.float32)
    yb = torch.from_numpy(y).to(torch.bfloat16).cuda()
    a = plan.backproject(yb, out_dtype=torch.bfloat16)
    a2 = plan.backproject(yb, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    assert torch.equal(a, a2)
    y_b = yb.double().cpu().numpy()
    check("H^T bf16", a.double().cpu().numpy(),
          ref.backproject(geom.as_dict(), y_b[rows], rows=rows), 2e-3, BF16_ELEM)
    p = torch.from_numpy(rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32))
    pb = p.to(torch.bfloat16).cuda()
    f = plan.fbp(pb, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    vox = rng.choice(geom.n_vox, 2000, replace=False)
    check("FBP bf16 voxels", f.double().cpu().numpy().ravel()[vox],
          ref.fbp(geom.as_dict(), pb.double().cpu().numpy(), voxels=vox), 2e-3, BF16_ELEM)
