"""Parity on the 256^3 / 8192-sphere-transducer plan (45 mm, 1024 samples)
with the library's default table budget, which holds its ~82 GB segment
table: the plan behind the reconstruction and time-to-residual
measurements.  64 windows of 128 transducers for G^T.

- H and G rows of transducers spread over the sphere;
- H^T for data on one transducer in every tenth window (the whole image);
- the adjoint identity with random x and y on all 8192 transducers.

Each comparison gates the relative L2 and max |error| / max |reference|.
"""
import sys

import numpy as np
import pytest

from checks import check
from paper_1304_2017_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from oracle import ref  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_sphere_8192_full_plan():
    from paper_1304_2017_amd.oat import Plan
    geom, _, img = synth.config_e(0)
    _say("[gpu-e] 256^3 / 8192 sphere transducers: building the plan")
    plan = Plan(geom, 0)
    try:
        st = plan.stats()
        _say(f"  segment table {st['segment_table_bytes'] / 1e9:.1f} GB")
        assert st["segment_table_bytes"] > 0
        gd = geom.as_dict()
        img64 = img.astype(np.float64)
        x = torch.from_numpy(img).cuda()
        p = plan.project(x)
        g = plan.project(x, srt_only=True)
        torch.cuda.synchronize()
        rows = np.array([0, 2731, 5000, 8191], dtype=np.int32)
        _say(f"[gpu-e] G and H rows {rows.tolist()}")
        check("G rows", g.double().cpu().numpy()[rows], ref.srt(gd, img64, rows=rows), 5e-7)
        check("H rows", p.double().cpu().numpy()[rows], ref.project(gd, img64, rows=rows), 1e-5)
        wins = np.arange(0, 64, 7)
        rows_t = np.array([w * 128 + (w * 37) % 128 for w in wins], dtype=np.int32)
        _say(f"[gpu-e] H^T with data on transducers {rows_t.tolist()}")
        rng = np.random.default_rng(16)
        y = np.zeros((geom.n_det, geom.n_t), dtype=np.float32)
        y[rows_t] = rng.normal(size=(rows_t.size, geom.n_t)).astype(np.float32)
        a = plan.backproject(torch.from_numpy(y).cuda())
        torch.cuda.synchronize()
        check("H^T", a.double().cpu().numpy(),
              ref.backproject(gd, y[rows_t].astype(np.float64), rows=rows_t), 1e-5)
        _say("[gpu-e] adjoint identity, random data on every transducer")
        gen = torch.Generator(device="cuda").manual_seed(17)
        xr = torch.randn(geom.shape, device="cuda", generator=gen)
        yr = torch.randn((geom.n_det, geom.n_t), device="cuda", generator=gen)
        Hx = plan.project(xr)
        HTy = plan.backproject(yr)
        torch.cuda.synchronize()
        lhs = float(torch.dot(Hx.double().ravel(), yr.double().ravel()))
        rhs = float(torch.dot(xr.double().ravel(), HTy.double().ravel()))
        scale = float(Hx.double().norm() * yr.double().norm())
        _say(f"  |<Hx,y> - <x,H^T y>| / (|Hx||y|) {abs(lhs - rhs) / scale:.3e}")
        assert abs(lhs - rhs) <= 1e-6 * scale
    finally:
        plan.close()
        torch.cuda.empty_cache()
