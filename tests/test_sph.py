"""Spherical-voxel imaging model H_sph (Sec. II.B.2, Eq. (dis_sph) with
Eq. (p0f)) and its adjoint (Eq. (sphbwd)), point-like transducers.

CPU: the oracle (oracle/ref.py) pinned to the Fourier transform of the
uniform-ball pressure, the small-f limit of p0, the adjoint identity and a
symmetry.  GPU: the library's H_sph and H_sph^T against the oracle.
"""
import sys

import numpy as np
import pytest
import torch  # before the library: one HIP runtime for both

from oracle import ref
from paper_1304_2017_amd import synth


def _geom1(d=20.0, dx=0.3, c0=1.5, gamma=1.7):
    return dict(nx=1, ny=1, nz=1, dx=dx, x0=0.0, y0=0.0, z0=0.0,
                det_xyz=np.array([[0.0, 0.0, d]]), det_area=None, n_t=64, dt=0.05, t0=0.0,
                c0=c0, gamma=gamma)


def test_one_voxel_is_the_spectrum_of_the_ball_pressure():
    """A single voxel of energy density A is a uniform ball of radius dx/2:
    its pressure at distance d is the N-wave (Gamma A / 2)(d - c0 t)/d for
    |c0 t - d| <= dx/2.  Its Fourier transform by quadrature must equal the
    model's output (reading: alpha_n is the voxel's energy density)."""
    g = _geom1()
    A = 0.7
    f = np.array([0.25, 1.0, 2.0, 3.7, 5.0, 9.0])
    got = np.array([ref.sph_project(g, np.full((1, 1, 1), A), 1, fi, 1.0)[0, 0] for fi in f])
    d, a, c0, gam = 20.0, 0.15, 1.5, 1.7
    t = np.linspace((d - a) / c0, (d + a) / c0, 400001)
    p = gam * A / 2 * (d - c0 * t) / d
    want = np.array([np.trapezoid(p * np.exp(-2j * np.pi * fi * t), t) for fi in f])
    assert np.max(np.abs(got - want)) < 1e-8 * np.max(np.abs(want))


def test_p0_small_frequency_limit():
    """Series of Eq. (p0f): p0(f) / f -> j Gamma pi^2 dx^3 / (6 c0^2) as f -> 0,
    and p0(0) = 0."""
    g = _geom1()
    lim = 1j * g["gamma"] * np.pi ** 2 * g["dx"] ** 3 / (6 * g["c0"] ** 2)
    f = np.array([1e-3, 1e-4])
    r = ref.sph_p0(f, g) / f
    assert np.all(np.abs(r - lim) < 1e-5 * abs(lim))
    assert ref.sph_p0(np.array([0.0]), g)[0] == 0


def test_sph_adjoint_identity():
    geom = synth.config_small(0)[0]
    gd = geom.as_dict()
    gd = dict(gd, nx=6, ny=5, nz=4)
    rng = np.random.default_rng(0)
    a = rng.normal(size=(4, 5, 6))
    n_f, f0, df = 12, 0.2, 0.31
    Q = gd["det_xyz"].shape[0]
    u = rng.normal(size=(Q, n_f)) + 1j * rng.normal(size=(Q, n_f))
    lhs = float(np.real(np.sum(np.conj(u) * ref.sph_project(gd, a, n_f, f0, df))))
    rhs = float(np.sum(a * ref.sph_backproject(gd, u, n_f, f0, df)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_voxel_at_the_centre_of_a_transducer_sphere():
    """Every transducer of a sphere sees the same spectrum from the centre
    voxel."""
    geom = synth.config_small(0)[0]
    gd = dict(geom.as_dict(), nx=1, ny=1, nz=1, x0=0.0, y0=0.0, z0=0.0)
    u = ref.sph_project(gd, np.ones((1, 1, 1)), 5, 0.5, 0.5)
    assert np.max(np.abs(u - u[0])) < 1e-13 * np.max(np.abs(u))


# --------------------------------------------------------------------------
# Finite transducer faces: the SIR as a surface integral over S_q
# --------------------------------------------------------------------------
def _face_geom():
    g = synth.config_small(0)[0].as_dict()
    return dict(g, nx=3, ny=4, nz=2)


def _frame(rq):
    d = np.linalg.norm(rq)
    t, p = np.arccos(rq[2] / d), np.arctan2(rq[1], rq[0])
    e1 = np.array([np.cos(t) * np.cos(p), np.cos(t) * np.sin(p), -np.sin(t)])
    e2 = np.array([np.sin(p), -np.cos(p), 0.0])
    return e1, e2, -rq / d


def test_sir_tends_to_the_point_transducer():
    """As the face shrinks, (1/S_q) h~_q tends to the point-like term."""
    g = _face_geom()
    r = np.array([[1.0, -2.0, 3.0], [0.0, 0.5, -4.0]])
    f = np.array([0.3, 2.0, 5.0])
    pt = ref.sph_sir(g, 7, r, f)
    small = ref.sph_sir(g, 7, r, f, aperture=(1e-4, 1e-4, 4))
    assert np.max(np.abs(small - pt)) <= 1e-7 * np.max(np.abs(pt))
    # and a 2 mm face differs from it at 5 MHz (the finite-aperture effect)
    big = ref.sph_sir(g, 7, r, f, aperture=(2.0, 2.0, 8))
    assert np.max(np.abs(big[2] - pt[2])) > 1e-2 * np.max(np.abs(pt[2]))


def test_sir_mirror_symmetries_of_the_face():
    """A rectangle centred on r_q is symmetric under a -> -a and b -> -b:
    sources mirrored across the planes (e3, e1) and (e3, e2) through r_q give
    equal responses."""
    g = _face_geom()
    q = 11
    rq = np.asarray(g["det_xyz"])[q]
    e1, e2, e3 = _frame(rq)
    base = rq + 20.0 * e3
    r = np.array([base + 1.3 * e1 + 0.7 * e2, base + 1.3 * e1 - 0.7 * e2,
                  base - 1.3 * e1 + 0.7 * e2])
    h = ref.sph_sir(g, q, r, np.array([1.0, 4.5]), aperture=(2.0, 1.5, 6))
    scale = np.max(np.abs(h))
    assert np.max(np.abs(h[:, 0] - h[:, 1])) <= 1e-13 * scale
    assert np.max(np.abs(h[:, 0] - h[:, 2])) <= 1e-13 * scale


def test_sir_on_axis_matches_the_radial_integral():
    """On the face's axis at distance z, with R = sqrt(z^2 + rho^2) and
    rho drho = R dR, the integral is
    (1/S) int_0^{2 pi} dphi/(2 pi) [exp(-j k z) - exp(-j k R_max(phi))] / (j k),
    R_max = sqrt(z^2 + rho_max^2), rho_max(phi) = min(w/(2|cos|), h/(2|sin|)):
    a 1-D integral done by adaptive quadrature, independent of the
    oracle's 2-D product rule."""
    from scipy.integrate import quad
    g = _face_geom()
    q = 3
    rq = np.asarray(g["det_xyz"])[q]
    _, _, e3 = _frame(rq)
    w, h, z = 2.0, 1.2, 17.0
    r = (rq + z * e3)[None, :]
    c0 = g["c0"]
    corner = np.arctan2(h, w)
    for f in (0.5, 3.0, 5.0):
        k = 2 * np.pi * f / c0

        def integrand(phi, part):
            c, s_ = abs(np.cos(phi)), abs(np.sin(phi))
            rho = min(w / (2 * c) if c > 0 else np.inf, h / (2 * s_) if s_ > 0 else np.inf)
            v = (np.exp(-1j * k * z) - np.exp(-1j * k * np.hypot(z, rho))) / (1j * k) / (2 * np.pi)
            return v.real if part == 0 else v.imag
        pts = [corner, np.pi - corner, np.pi + corner, 2 * np.pi - corner]
        want = sum(quad(integrand, 0, 2 * np.pi, args=(i,), points=pts, epsabs=0,
                        epsrel=1e-13, limit=200)[0] * (1j if i else 1) for i in (0, 1)) / (w * h)
        got = ref.sph_sir(g, q, r, [f], aperture=(w, h, 20))[0, 0]
        assert abs(got - want) <= 1e-10 * abs(want), (f, got, want)


def test_sph_adjoint_identity_with_faces():
    g = _face_geom()
    rng = np.random.default_rng(5)
    a = rng.normal(size=(2, 4, 3))
    n_f, f0, df = 6, 0.4, 0.7
    Q = np.asarray(g["det_xyz"]).shape[0]
    u = rng.normal(size=(Q, n_f)) + 1j * rng.normal(size=(Q, n_f))
    ap = (2.0, 2.0, 3)
    lhs = float(np.real(np.sum(np.conj(u) * ref.sph_project(g, a, n_f, f0, df, aperture=ap))))
    rhs = float(np.sum(a * ref.sph_backproject(g, u, n_f, f0, df, aperture=ap)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# --------------------------------------------------------------------------
# The library's H_sph and H_sph^T against the oracle (GPU)
# --------------------------------------------------------------------------
gpu = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _small_geom(nx=12, ny=10, nz=8):
    g = synth.config_small(0)[0]
    return synth.Geometry(nx, ny, nz, g.dx, synth.centred_origin(nx, g.dx),
                          synth.centred_origin(ny, g.dx), synth.centred_origin(nz, g.dx),
                          g.det_xyz, g.n_t, g.dt, g.t0, g.c0, 1.3)


@pytest.fixture(scope="module")
def small_sph():
    from paper_1304_2017_amd.oat import Plan
    geom = _small_geom()
    return geom, Plan(geom, 0)


@gpu
@pytest.mark.parametrize("n_f,f0,df", [(40, 0.1, 0.1), (7, 0.0, 0.35), (130, 0.02, 0.038)])
def test_sph_project_and_backproject(small_sph, n_f, f0, df):
    geom, plan = small_sph
    gd = geom.as_dict()
    rng = np.random.default_rng(n_f)
    a = rng.uniform(0, 1, size=geom.shape).astype(np.float32).astype(np.float64)
    a[rng.uniform(size=geom.shape) < 0.3] = 0.0          # some empty voxels
    u = plan.sph_project(torch.from_numpy(a).float().cuda(), n_f, f0, df)
    u2 = plan.sph_project(torch.from_numpy(a).float().cuda(), n_f, f0, df)
    torch.cuda.synchronize()
    e = rel(u.cpu().numpy(), ref.sph_project(gd, a, n_f, f0, df))
    y = (rng.normal(size=(geom.n_det, n_f)) + 1j * rng.normal(size=(geom.n_det, n_f)))
    y = y.astype(np.complex64)
    b = plan.sph_backproject(torch.from_numpy(y).cuda(), f0, df)
    torch.cuda.synchronize()
    eT = rel(b.double().cpu().numpy(), ref.sph_backproject(gd, y.astype(np.complex128), n_f, f0, df))
    # adjoint identity through the library, scaled by the norms
    uy = torch.from_numpy(y).cuda()
    lhs = float(torch.real(torch.sum(torch.conj(uy.to(torch.complex128)) * u.to(torch.complex128))))
    rhs = float(torch.sum(torch.from_numpy(a).cuda() * plan.sph_backproject(uy, f0, df).double()))
    scale = float(u.abs().double().norm() * uy.abs().double().norm())
    _say(f"[gpu] H_sph n_f {n_f}: rel {e:.3e}  H_sph^T rel {eT:.3e}  "
         f"adjoint {abs(lhs - rhs) / scale:.3e}")
    assert e < 1e-5 and eT < 1e-5
    assert abs(lhs - rhs) <= 1e-5 * scale
    assert torch.equal(u, u2)


@gpu
def test_sph_bf16_image(small_sph):
    geom, plan = small_sph
    rng = np.random.default_rng(3)
    ab = torch.from_numpy(rng.uniform(0, 1, size=geom.shape)).to(torch.bfloat16)
    u = plan.sph_project(ab.cuda(), 16, 0.2, 0.2)
    torch.cuda.synchronize()
    e = rel(u.cpu().numpy(), ref.sph_project(geom.as_dict(), ab.double().numpy(), 16, 0.2, 0.2))
    y = torch.from_numpy((rng.normal(size=(geom.n_det, 16)) + 1j * rng.normal(size=(geom.n_det, 16)))
                         .astype(np.complex64)).cuda()
    b = plan.sph_backproject(y, 0.2, 0.2, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    eb = rel(b.double().cpu().numpy(),
             ref.sph_backproject(geom.as_dict(), y.cpu().numpy().astype(np.complex128), 16, 0.2, 0.2))
    _say(f"[gpu] H_sph BF16 image rel {e:.3e}; H_sph^T BF16 output rel {eb:.3e}")
    assert e < 1e-5 and eb < 2e-3


@gpu
def test_sph_arguments(small_sph):
    from paper_1304_2017_amd import oat
    geom, plan = small_sph
    L = oat.lib()
    x = torch.zeros(geom.shape, device="cuda")
    u = torch.zeros((geom.n_det, 4), device="cuda", dtype=torch.complex64)
    vp = oat.ctypes.c_void_p
    assert L.oat_sph_project(plan._h, vp(x.data_ptr()), 0, vp(u.data_ptr()), 0, 0.0, 1.0, 0,
                             None) == oat.OAT_ERR_ARG
    assert L.oat_sph_project(plan._h, vp(x.data_ptr()), 0, vp(u.data_ptr()), 4, 0.0, -1.0, 0,
                             None) == oat.OAT_ERR_ARG
    assert L.oat_sph_backproject(plan._h, vp(u.data_ptr()), 4, 0.0, 1.0, vp(x.data_ptr()), 5, 0,
                                 None) == oat.OAT_ERR_DTYPE
    big = torch.zeros((geom.n_det, 4097), device="cuda", dtype=torch.complex64)
    assert L.oat_sph_project(plan._h, vp(x.data_ptr()), 0, vp(big.data_ptr()), 4097, 0.0, 1.0, 0,
                             None) == oat.OAT_ERR_ARG


@gpu
def test_sph_largest_frequency_count(small_sph):
    """n_f = 4096, the largest accepted: one workgroup holds a transducer's
    frequency blocks."""
    geom, plan = small_sph
    rng = np.random.default_rng(11)
    a = np.zeros(geom.shape)
    a[rng.uniform(size=geom.shape) < 0.05] = 1.0
    u = plan.sph_project(torch.from_numpy(a).float().cuda(), 4096, 0.0, 0.002)
    torch.cuda.synchronize()
    rows = np.array([0, 37])
    e = rel(u.cpu().numpy()[rows], ref.sph_project(geom.as_dict(), a, 4096, 0.0, 0.002, rows=rows))
    _say(f"[gpu] H_sph n_f 4096: rel {e:.3e}")
    assert e < 1e-5


@gpu
def test_sph_at_64cube_2048_rows_and_voxels():
    """64^3 at 0.4 mm, 2048 hemisphere transducers, 256 frequencies in
    (0, 5] MHz (the benchmark's shape): sampled rows of H_sph and sampled
    voxels of H_sph^T against the oracle."""
    from paper_1304_2017_amd.oat import Plan
    geom, img = synth.config_sph()
    plan = Plan(geom, 0)
    n_f, df = 256, 5.0 / 256
    gd = geom.as_dict()
    u = plan.sph_project(torch.from_numpy(img).float().cuda(), n_f, df, df)
    torch.cuda.synchronize()
    rows = np.array([0, 1023, 2047])
    e = rel(u.cpu().numpy()[rows], ref.sph_project(gd, img.astype(np.float64), n_f, df, df, rows=rows))
    rng = np.random.default_rng(4)
    y = (rng.normal(size=(geom.n_det, n_f)) + 1j * rng.normal(size=(geom.n_det, n_f))).astype(np.complex64)
    b = plan.sph_backproject(torch.from_numpy(y).cuda(), df, df)
    torch.cuda.synchronize()
    vox = rng.choice(geom.n_vox, 40, replace=False)
    eT = rel(b.double().cpu().numpy().ravel()[vox],
             ref.sph_backproject(gd, y.astype(np.complex128), n_f, df, df, voxels=vox))
    _say(f"[gpu-full] H_sph 64^3/2048/256 rows rel {e:.3e}; H_sph^T voxels rel {eT:.3e}")
    assert e < 1e-5 and eT < 1e-5


@gpu
def test_sph_adjoint_without_slices():
    """An image of 128 x 64 x 64 = 2^19 voxels fills 1024 workgroups, so the
    adjoint takes all transducers in one pass and stores directly (smaller
    images split them into slices of FP64 partial images): sampled voxels
    against the oracle, and the adjoint identity on the whole image."""
    from paper_1304_2017_amd.oat import Plan
    nx, ny, nz, dx = 128, 64, 64, 0.4
    geom = synth.Geometry(nx, ny, nz, dx, synth.centred_origin(nx, dx), synth.centred_origin(ny, dx),
                          synth.centred_origin(nz, dx), synth.fibonacci_sphere(48, 40.0), 256, 0.05,
                          0.0, 1.5, 1.0)
    assert geom.n_vox == 1 << 19
    plan = Plan(geom, 0, arc_table=False, segment_table=False)
    n_f, f0, df = 24, 0.2, 0.2
    gd = geom.as_dict()
    rng = np.random.default_rng(8)
    y = (rng.normal(size=(geom.n_det, n_f)) + 1j * rng.normal(size=(geom.n_det, n_f))).astype(np.complex64)
    b = plan.sph_backproject(torch.from_numpy(y).cuda(), f0, df)
    x = torch.from_numpy(rng.uniform(0, 1, size=geom.shape).astype(np.float32)).cuda()
    u = plan.sph_project(x, n_f, f0, df)
    torch.cuda.synchronize()
    vox = rng.choice(geom.n_vox, 60, replace=False)
    eT = rel(b.double().cpu().numpy().ravel()[vox],
             ref.sph_backproject(gd, y.astype(np.complex128), n_f, f0, df, voxels=vox))
    lhs = float(np.real(np.vdot(y.astype(np.complex128), u.cpu().numpy().astype(np.complex128))))
    rhs = float(np.dot(x.double().cpu().numpy().ravel(), b.double().cpu().numpy().ravel()))
    scale = float(np.linalg.norm(u.cpu().numpy()) * np.linalg.norm(y))
    _say(f"[gpu] H_sph^T 128x64x64 (one slice) voxels rel {eT:.3e}; "
         f"adjoint {abs(lhs - rhs) / scale:.3e}")
    assert eT < 1e-5
    assert abs(lhs - rhs) <= 1e-5 * scale


@gpu
@pytest.mark.parametrize("ap", [(2.0, 2.0, 4), (2.0, 1.2, 3), (0.5, 0.5, 1)])
def test_sph_finite_faces(ap):
    """H_sph and H_sph^T with flat rectangular faces (m x m Gauss-Legendre
    nodes) against the oracle's face quadrature, the adjoint identity, and
    the return to point-like transducers."""
    from paper_1304_2017_amd.oat import Plan
    geom = _small_geom()
    plan = Plan(geom, 0, arc_table=False, segment_table=False)
    gd = geom.as_dict()
    n_f, f0, df = 40, 0.1, 0.12
    rng = np.random.default_rng(int(ap[2]) * 10 + int(ap[1] * 10))
    a = rng.uniform(0, 1, size=geom.shape).astype(np.float32).astype(np.float64)
    a[rng.uniform(size=geom.shape) < 0.3] = 0.0
    plan.set_aperture(*ap)
    x = torch.from_numpy(a).float().cuda()
    u = plan.sph_project(x, n_f, f0, df)
    y = (rng.normal(size=(geom.n_det, n_f)) + 1j * rng.normal(size=(geom.n_det, n_f)))
    y = y.astype(np.complex64)
    yd = torch.from_numpy(y).cuda()
    b = plan.sph_backproject(yd, f0, df)
    torch.cuda.synchronize()
    e = rel(u.cpu().numpy(), ref.sph_project(gd, a, n_f, f0, df, aperture=ap))
    eT = rel(b.double().cpu().numpy(),
             ref.sph_backproject(gd, y.astype(np.complex128), n_f, f0, df, aperture=ap))
    lhs = float(np.real(np.vdot(y.astype(np.complex128), u.cpu().numpy().astype(np.complex128))))
    rhs = float(np.dot(a.ravel(), b.double().cpu().numpy().ravel()))
    scale = float(np.linalg.norm(u.cpu().numpy()) * np.linalg.norm(y))
    # the faces change the model: compare with point-like transducers
    plan.set_aperture(0.0, 0.0)
    u0 = plan.sph_project(x, n_f, f0, df)
    torch.cuda.synchronize()
    e0 = rel(u0.cpu().numpy(), ref.sph_project(gd, a, n_f, f0, df))
    d0 = rel(u.cpu().numpy(), u0.cpu().numpy())
    _say(f"[gpu] H_sph faces {ap}: rel {e:.3e}, H_sph^T rel {eT:.3e}, adjoint "
         f"{abs(lhs - rhs) / scale:.3e}; point-like again rel {e0:.3e} (faces vs point {d0:.2e})")
    assert e < 1e-5 and eT < 1e-5 and e0 < 1e-5
    assert abs(lhs - rhs) <= 1e-5 * scale
    if ap[2] == 1:
        assert d0 == 0.0      # one Gauss node is the face centre: the point-like model
    else:
        assert d0 > 1e-4


@gpu
def test_sph_faces_without_slices_and_arguments():
    """Faces on the single-pass adjoint (2^19 voxels, no slices): sampled
    voxels against the oracle; and the argument checks."""
    from paper_1304_2017_amd import oat
    from paper_1304_2017_amd.oat import Plan
    nx, ny, nz, dx = 128, 64, 64, 0.4
    geom = synth.Geometry(nx, ny, nz, dx, synth.centred_origin(nx, dx), synth.centred_origin(ny, dx),
                          synth.centred_origin(nz, dx), synth.fibonacci_sphere(48, 40.0), 256, 0.05,
                          0.0, 1.5, 1.0)
    plan = Plan(geom, 0, arc_table=False, segment_table=False)
    L = oat.lib()
    assert L.oat_plan_set_aperture(plan._h, -1.0, 1.0, 2) == oat.OAT_ERR_ARG
    assert L.oat_plan_set_aperture(plan._h, 1.0, 0.0, 2) == oat.OAT_ERR_ARG
    assert L.oat_plan_set_aperture(plan._h, 1.0, 1.0, 0) == oat.OAT_ERR_ARG
    assert L.oat_plan_set_aperture(plan._h, 1.0, 1.0, 9) == oat.OAT_ERR_ARG
    assert L.oat_plan_set_aperture(plan._h, 30.0, 30.0, 2) == oat.OAT_ERR_GEOMETRY
    ap = (2.0, 2.0, 2)
    plan.set_aperture(*ap)
    n_f, f0, df = 24, 0.2, 0.2
    rng = np.random.default_rng(9)
    y = (rng.normal(size=(geom.n_det, n_f)) + 1j * rng.normal(size=(geom.n_det, n_f))).astype(np.complex64)
    b = plan.sph_backproject(torch.from_numpy(y).cuda(), f0, df)
    torch.cuda.synchronize()
    vox = rng.choice(geom.n_vox, 40, replace=False)
    eT = rel(b.double().cpu().numpy().ravel()[vox],
             ref.sph_backproject(geom.as_dict(), y.astype(np.complex128), n_f, f0, df, voxels=vox,
                                 aperture=ap))
    _say(f"[gpu] H_sph^T faces 128x64x64 (one slice) voxels rel {eT:.3e}")
    assert eT < 1e-5
