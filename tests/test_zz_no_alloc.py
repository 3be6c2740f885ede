"""oat_sph_backproject_noalloc: the spherical-voxel adjoint (Eq. (sphbwd))
through the entry point that allocates nothing, whose slice partial images go
to the library's fixed per-GPU scratch.  Checked through the C ABI against
oat_sph_backproject (bit for bit: same kernels, same order of sums) and, on
sampled voxels, against the FP64 oracle, on two calls in a row, the second on
a smaller image with fewer frequencies."""
import ctypes
import sys

import numpy as np
import pytest
import torch  # before the library: one HIP runtime for both

from oracle import ref
from paper_1304_2017_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _geom(nx, ny, nz, n_det, dx=0.4):
    return synth.Geometry(nx, ny, nz, dx, synth.centred_origin(nx, dx),
                          synth.centred_origin(ny, dx), synth.centred_origin(nz, dx),
                          synth.fibonacci_sphere(n_det, 40.0), 256, 0.05, 0.0, 1.5, 1.3)


def _case(geom, n_f, f0, df, seed):
    from paper_1304_2017_amd import oat
    from paper_1304_2017_amd.oat import Plan
    L = oat.lib()
    plan = Plan(geom, 0, arc_table=False, segment_table=False)
    rng = np.random.default_rng(seed)
    y = (rng.normal(size=(geom.n_det, n_f)) + 1j * rng.normal(size=(geom.n_det, n_f)))
    y = y.astype(np.complex64)
    yd = torch.from_numpy(y).cuda()
    out = torch.full(geom.shape, float("nan"), device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    _say(f"[gpu] noalloc case {geom.shape} n_f {n_f} seed {seed}")
    rc = L.oat_sph_backproject_noalloc(plan._h, ctypes.c_void_p(yd.data_ptr()), n_f, float(f0),
                                       float(df), ctypes.c_void_p(out.data_ptr()), oat.OAT_F32, 0,
                                       None)
    assert rc == oat.OAT_OK, oat.last_error()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    want = plan.sph_backproject(yd, f0, df)
    torch.cuda.synchronize()
    vox = rng.choice(geom.n_vox, 40, replace=False)
    e = float(np.linalg.norm(out.double().cpu().numpy().ravel()[vox]
                             - ref.sph_backproject(geom.as_dict(), y.astype(np.complex128), n_f,
                                                   f0, df, voxels=vox))
              / np.linalg.norm(ref.sph_backproject(geom.as_dict(), y.astype(np.complex128), n_f,
                                                   f0, df, voxels=vox)))
    same = torch.equal(out, want)
    _say(f"[gpu] noalloc {geom.shape}: bit-identical to oat_sph_backproject {same}; "
         f"sampled voxels rel {e:.3e} vs the oracle")
    assert same
    assert e < 1e-5
    plan.close()


def test_noalloc_matches_the_allocating_adjoint_twice():
    # 46080 voxels: four transducer slices in the scratch
    _case(_geom(40, 36, 32, 64), 48, 0.1, 0.15, 1)
    # then a smaller image and fewer frequencies on the same scratch
    _case(_geom(12, 10, 8, 24), 20, 0.0, 0.3, 2)


def test_noalloc_rejects_bad_arguments():
    from paper_1304_2017_amd import oat
    from paper_1304_2017_amd.oat import Plan
    L = oat.lib()
    geom = _geom(12, 10, 8, 24)
    plan = Plan(geom, 0, arc_table=False, segment_table=False)
    x = torch.zeros(geom.shape, device="cuda")
    u = torch.zeros((geom.n_det, 4), device="cuda", dtype=torch.complex64)
    vp = ctypes.c_void_p
    assert L.oat_sph_backproject_noalloc(plan._h, vp(u.data_ptr()), 0, 0.0, 1.0,
                                         vp(x.data_ptr()), 0, 0, None) == oat.OAT_ERR_ARG
    assert L.oat_sph_backproject_noalloc(plan._h, vp(u.data_ptr()), 4, 0.0, 1.0,
                                         vp(x.data_ptr()), 7, 0, None) == oat.OAT_ERR_DTYPE
    assert L.oat_sph_backproject_noalloc(plan._h, vp(u.data_ptr()), 4, 0.0, 1.0,
                                         vp(u.data_ptr()), 0, 0, None) == oat.OAT_ERR_ARG
    plan.close()
