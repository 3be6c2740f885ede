"""Transducer electrical impulse response (EIR): H^e of Eq. (EIR), its
adjoint (Sec. II.B.3), and the Hann-window Fourier deconvolution applied
before FBP (Sec. IV.B).

CPU: the oracle (oracle/ref.py) pinned to closed forms, a library
convolution and FFT, the adjoint identity, and the paper's printed
simulation setup (tests/golden/paper_simulation_setup.json).
GPU: the library's EIR paths against the oracle.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch  # before the library: one HIP runtime for both

from oracle import ref
from paper_1304_2017_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_simulation_setup.json")


gamma_pulse = synth.gamma_pulse


# --------------------------------------------------------------------------
# Oracle pins (CPU)
# --------------------------------------------------------------------------
def test_eir_single_tap_is_a_one_sample_delay():
    p = np.random.default_rng(0).normal(size=(3, 17))
    u = ref.eir([1.0], p)
    assert np.array_equal(u[:, 0], np.zeros(3))
    assert np.array_equal(u[:, 1:], p[:, :-1])


def test_eir_matches_a_library_convolution():
    rng = np.random.default_rng(1)
    h = rng.normal(size=7)
    p = rng.normal(size=(2, 40))
    u = ref.eir(h, p)
    for q in range(2):
        full = np.convolve(h, p[q])          # full[n] = sum_m h[m] p[n - m]
        want = np.concatenate([[0.0], full[:39]])
        assert np.allclose(u[q], want, rtol=0, atol=1e-13)


def test_eir_impulse_response_is_the_delayed_taps():
    h = np.array([0.5, -1.0, 2.0, 0.25])
    p = np.zeros((1, 12))
    p[0, 3] = 1.0
    u = ref.eir(h, p)[0]
    want = np.zeros(12)
    want[4:8] = h
    assert np.array_equal(u, want)


def test_eir_adjoint_identity():
    rng = np.random.default_rng(2)
    h = rng.normal(size=9)
    p = rng.normal(size=(4, 50))
    u = rng.normal(size=(4, 50))
    lhs = float(np.sum(ref.eir(h, p) * u))
    rhs = float(np.sum(p * ref.eir_adj(h, u)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.array_equal(ref.eir_matrix(h, 50).T, _adj_matrix(h, 50))


def _adj_matrix(h, K):
    """The adjoint formula written out element by element (brute force)."""
    A = np.zeros((K, K))
    for k in range(K):
        for kappa in range(K):
            m = kappa - 1 - k
            if 0 <= m < len(h):
                A[k, kappa] = h[m]
    return A


def test_hann_window_closed_forms():
    fc = 5.0
    w = ref.hann(np.array([0.0, 2.5, 5.0, 5.5, -2.5, -7.0, 1.25]), fc)
    assert w[0] == 1.0 and abs(w[1] - 0.5) < 1e-15 and w[2] == 0.0 and w[3] == 0.0
    assert w[4] == w[1] and w[5] == 0.0
    assert abs(w[6] - (1 - np.cos(np.pi * 0.75)) / 2) < 1e-15


def test_deconvolution_undoes_the_eir_up_to_the_window():
    """For a record whose full convolution fits in K samples, deconvolving
    H^e p gives p filtered by the window alone: IFFT(W FFT(p))."""
    K, dt, fc = 256, 0.05, 5.0
    h = gamma_pulse(24, dt, 0.08)
    rng = np.random.default_rng(3)
    p = np.zeros((3, K))
    p[:, :K // 2] = rng.normal(size=(3, K // 2))
    got = ref.deconvolve(h, ref.eir(h, p), dt, fc)
    N = ref.deconv_length(K)
    want = np.fft.ifft(np.fft.fft(p, n=N, axis=-1) * ref.hann(np.fft.fftfreq(N, dt), fc),
                       axis=-1).real[:, :K]
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))


def test_deconvolution_of_a_sinusoid_in_the_band():
    """A unit-delay EIR and a sinusoid on the FFT grid well inside the
    record: the result is W(f0) times the sinusoid away from the ends."""
    K, dt, fc = 512, 0.05, 5.0
    N = ref.deconv_length(K)
    f0 = 40 / (N * dt)                        # 1.95 MHz, on the grid
    t = np.arange(K) * dt
    p = np.sin(2 * np.pi * f0 * t)[None, :]
    got = ref.deconvolve([1.0], ref.eir([1.0], p), dt, fc)
    # the record is finite, so compare against the windowed transform of
    # the zero-padded record; in the middle third it is close to W(f0) p
    mid = slice(K // 3, 2 * K // 3)
    assert np.max(np.abs(got[0, mid] - ref.hann(f0, fc) * p[0, mid])) < 0.05


def test_paper_simulation_setup():
    """The paper's printed simulation parameters, their internal consistency,
    and the 210x210x440 workload built from them."""
    g = json.load(open(GOLDEN))
    # printed grid and phantom cuboid agree: nodes x spacing
    for n, L in zip(g["grid_nodes"], g["phantom_cuboid_mm"]):
        assert abs(n * g["grid_spacing_mm"] - L) < 1e-9
    # 128 rings over the full polar angle with theta_min = pi/256: mid-band rings
    assert abs(0.5 / g["rings_full"] - g["theta_min_full_rad_over_pi"]) < 1e-15
    # 511 spectral components in (0, 5] MHz: bins of width fs / (2K)
    K, fs = g["samples_per_transducer"], g["sampling_rate_mhz"]
    df = fs / (2 * K)
    assert int(np.floor(g["hann_cutoff_mhz"] / df + 1e-9)) == g["spectral_components_in_0_to_5_mhz"]
    # the 64x90 workload
    geom = synth.config_p_geometry()
    assert (geom.nx, geom.ny, geom.nz) == tuple(g["grid_nodes"])
    assert abs(geom.dx - g["grid_spacing_mm"]) < 1e-12
    assert abs(geom.c0 - g["speed_of_sound_mm_per_us"]) < 1e-12
    assert geom.n_t == K and abs(geom.dt - 1.0 / fs) < 1e-12
    assert geom.n_det == g["subset_rings"] * g["views"]
    r = np.linalg.norm(geom.det_xyz, axis=1)
    assert np.allclose(r, g["measurement_sphere_radius_mm"])
    theta = np.arccos(np.clip(geom.det_xyz[:, 2] / r, -1, 1))
    rings = np.unique(np.round(theta, 9))
    assert rings.size == g["subset_rings"]
    assert np.allclose(rings, (np.arange(g["subset_rings"]) + 0.5) * np.pi / g["subset_rings"])


# --------------------------------------------------------------------------
# The library's EIR paths against the oracle (GPU)
# --------------------------------------------------------------------------
gpu = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _t(x, dtype=None):
    import torch
    return torch.tensor(np.asarray(x), dtype=torch.float64).to(dtype or torch.float32).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.fixture(scope="module")
def small_eir():
    from paper_1304_2017_amd.oat import Plan
    geom = synth.config_small(0)[0]
    plan = Plan(geom, 0)
    h = gamma_pulse(24, geom.dt, 0.3)
    plan.set_eir(h)
    return geom, plan, h


@gpu
def test_project_and_backproject_with_eir(small_eir):
    import torch
    geom, plan, h = small_eir
    gd = geom.as_dict()
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 1, size=geom.shape).astype(np.float32).astype(np.float64)
    _say("[gpu] H and H^T with a 24-tap EIR, 32^3")
    e = rel(_np(plan.project(_t(img))), ref.project_eir(gd, h, img))
    y = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32).astype(np.float64)
    eT = rel(_np(plan.backproject(_t(y))), ref.backproject_eir(gd, h, y))
    # G alone is unchanged by the EIR
    eg = rel(_np(plan.project(_t(img), srt_only=True)), ref.srt(gd, img))
    # adjoint identity through the library
    x = _t(img, torch.float64).float()
    yy = _t(y, torch.float64).float()
    Hx = plan.project(x).double()
    lhs = float((Hx * yy.double()).sum())
    rhs = float((x.double() * plan.backproject(yy).double()).sum())
    scale = float(Hx.norm() * yy.double().norm())
    _say(f"  H rel {e:.3e}  H^T rel {eT:.3e}  G rel {eg:.3e}  "
         f"|<Hx,y>-<x,H^T y>| / (|Hx||y|) {abs(lhs - rhs) / scale:.3e}")
    assert e < 1e-5 and eT < 1e-5 and eg < 1e-6
    assert abs(lhs - rhs) <= 1e-5 * scale


@gpu
def test_eir_with_bf16_storage(small_eir):
    import torch
    geom, plan, h = small_eir
    gd = geom.as_dict()
    rng = np.random.default_rng(6)
    img = rng.uniform(0, 1, size=geom.shape)
    xb = _t(img, torch.bfloat16)
    e = rel(_np(plan.project(xb, out_dtype=torch.bfloat16)), ref.project_eir(gd, h, _np(xb)))
    _say(f"[gpu] H with EIR, BF16 storage: rel {e:.3e}")
    assert e < 2e-3


@gpu
def test_deconvolve_matches_oracle(small_eir):
    import torch
    geom, plan, h = small_eir
    rng = np.random.default_rng(7)
    u = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32).astype(np.float64)
    fc = 2.5                                   # MHz; sampling at 10 MHz
    p = plan.deconvolve(_t(u), fc)
    p2 = plan.deconvolve(_t(u), fc)
    e = rel(_np(p), ref.deconvolve(h, u, geom.dt, fc))
    _say(f"[gpu] deconvolution rel {e:.3e}")
    assert e < 1e-6
    assert torch.equal(p, p2)
    ub = _t(u, torch.bfloat16)
    eb = rel(_np(plan.deconvolve(ub, fc, out_dtype=torch.bfloat16)),
             ref.deconvolve(h, _np(ub), geom.dt, fc))
    assert eb < 2e-3


@gpu
def test_deconvolution_then_fbp(small_eir):
    """FBP of deconvolved EIR-filtered data, against the oracle's
    deconvolution and FBP."""
    geom, plan, h = small_eir
    gd = geom.as_dict()
    _, balls, _ = synth.config_small(0)
    p_true = synth.nwave_balls(geom, balls)
    u = ref.eir(h, p_true).astype(np.float32).astype(np.float64)
    got = _np(plan.fbp(plan.deconvolve(_t(u), 2.5)))
    want = ref.fbp(gd, ref.deconvolve(h, u, geom.dt, 2.5))
    e = rel(got, want)
    _say(f"[gpu] deconvolution + FBP rel {e:.3e}")
    assert e < 1e-5


@gpu
def test_eir_arguments_and_removal(small_eir):
    from paper_1304_2017_amd import oat
    geom, plan, h = small_eir
    L = oat.lib()
    too_many = np.zeros(geom.n_t + 1)
    dp = too_many.ctypes.data_as(oat.ctypes.POINTER(oat.ctypes.c_double))
    assert L.oat_plan_set_eir(plan._h, dp, geom.n_t + 1) == oat.OAT_ERR_ARG
    bad = np.array([1.0, np.nan])
    assert L.oat_plan_set_eir(plan._h, bad.ctypes.data_as(oat.ctypes.POINTER(oat.ctypes.c_double)),
                              2) == oat.OAT_ERR_ARG
    u = _t(np.zeros((geom.n_det, geom.n_t)))
    with pytest.raises(oat.OatError):
        plan.deconvolve(u, 0.0)
    # removing the EIR restores H = D G, and deconvolution then refuses
    rng = np.random.default_rng(8)
    img = rng.uniform(0, 1, size=geom.shape).astype(np.float32).astype(np.float64)
    plan.set_eir(None)
    try:
        assert rel(_np(plan.project(_t(img))), ref.project(geom.as_dict(), img)) < 1e-5
        with pytest.raises(oat.OatError):
            plan.deconvolve(u, 2.5)
    finally:
        plan.set_eir(h)


@gpu
def test_full_size_eir_rows():
    """256^3 / 2048 / 1024 with a 64-tap EIR: H on sampled rows, H^T with
    data on two transducers, and the deconvolution of every row."""
    import torch
    from paper_1304_2017_amd.oat import Plan
    geom, _, img = synth.config_large(0, dtype=np.float32)
    plan = Plan(geom, 0)
    h = gamma_pulse(64, geom.dt, 0.1)
    plan.set_eir(h)
    gd = geom.as_dict()
    rows = np.array([5, 1400], dtype=np.int32)
    _say("[gpu-full] H with EIR, rows 5 and 1400")
    p = _np(plan.project(torch.from_numpy(img).cuda()))
    e = rel(p[rows], ref.project_eir(gd, h, img.astype(np.float64), rows=rows))
    y = np.zeros((geom.n_det, geom.n_t), dtype=np.float32)
    y[rows] = np.random.default_rng(9).normal(size=(2, geom.n_t)).astype(np.float32)
    a = _np(plan.backproject(torch.from_numpy(y).cuda()))
    eT = rel(a, ref.backproject_eir(gd, h, y[rows].astype(np.float64), rows=rows))
    u = np.random.default_rng(10).normal(size=(geom.n_det, geom.n_t)).astype(np.float32)
    d = _np(plan.deconvolve(torch.from_numpy(u).cuda(), 5.0))
    ed = rel(d, ref.deconvolve(h, u.astype(np.float64), geom.dt, 5.0))
    _say(f"  H rel {e:.3e}  H^T rel {eT:.3e}  deconvolution rel {ed:.3e}")
    assert e < 1e-5 and eT < 1e-5 and ed < 1e-6
