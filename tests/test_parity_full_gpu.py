"""Parity at the full benchmark size (256^3 nodes at 0.1 mm, 2048 transducers,
1024 samples), in the launch configuration bench.py times, on outputs the
FP64 oracle can compute one by one:

- H and G: whole rows of a few transducers (the oracle evaluates rows);
- H^T: the full image for data that is nonzero on two transducers only
  (the kernel still walks every transducer's points);
- FBP: sampled voxels of the full image for seeded Gaussian data.
"""
import sys

import numpy as np
import pytest

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
    eg = rel(g, ref.srt(gd, img64, rows=rows))
    ep = rel(p, ref.project(gd, img64, rows=rows))
    _say(f"  G rel {eg:.3e}  H rel {ep:.3e}")
    assert eg < 1e-6
    assert ep < 1e-5


def test_full_size_project_rows_bf16(large):
    geom, img, plan = large
    rows = np.array([333, 1777], dtype=np.int32)
    _say("[gpu-full] H BF16")
    xb = torch.from_numpy(img).to(torch.bfloat16).cuda()
    p = plan.project(xb, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    p = p.double().cpu().numpy()[rows]
    img_b = xb.double().cpu().numpy()
    e = rel(p, ref.project(geom.as_dict(), img_b, rows=rows))
    _say(f"  rel {e:.3e}")
    assert e < 2e-3


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
    e = rel(a, want)
    _say(f"  rel {e:.3e}")
    assert e < 1e-5


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
    e = rel(f[vox], want)
    _say(f"  rel {e:.3e}")
    assert e < 1e-5


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
    eh = rel(p, ref.project(gd, img64))
    rng = np.random.default_rng(21)
    y = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32)
    a = plan.backproject(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    eht = rel(a.double().cpu().numpy(), ref.backproject(gd, y.astype(np.float64)))
    pf = p.astype(np.float32)
    f = plan.fbp(torch.from_numpy(pf).cuda())
    torch.cuda.synchronize()
    ef = rel(f.double().cpu().numpy(), ref.fbp(gd, pf.astype(np.float64)))
    _say(f"  H rel {eh:.3e}  H^T rel {eht:.3e}  FBP rel {ef:.3e}")
    assert eh < 1e-5 and eht < 1e-5 and ef < 1e-5


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
    eg = rel(g.double().cpu().numpy()[rows], ref.srt(gd, img64, rows=rows))
    ep = rel(p.double().cpu().numpy()[rows], ref.project(gd, img64, rows=rows))
    pn = p.float()
    f = plan.fbp(pn)
    torch.cuda.synchronize()
    vox = np.random.default_rng(22).choice(geom.n_vox, 2000, replace=False)
    ef = rel(f.double().cpu().numpy().ravel()[vox],
             ref.fbp(gd, pn.double().cpu().numpy(), voxels=vox))
    _say(f"  G rel {eg:.3e}  H rel {ep:.3e}  FBP rel {ef:.3e}")
    assert eg < 1e-6 and ep < 1e-5 and ef < 1e-5


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
    e = rel(a.double().cpu().numpy(), ref.backproject(geom.as_dict(), y_b[rows], rows=rows))
    p = torch.from_numpy(rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32))
    pb = p.to(torch.bfloat16).cuda()
    f = plan.fbp(pb, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    vox = rng.choice(geom.n_vox, 2000, replace=False)
    ef = rel(f.double().cpu().numpy().ravel()[vox],
             ref.fbp(geom.as_dict(), pb.double().cpu().numpy(), voxels=vox))
    _say(f"[gpu-full] BF16 H^T rel {e:.3e}  FBP rel {ef:.3e}")
    assert e < 2e-3 and ef < 2e-3
