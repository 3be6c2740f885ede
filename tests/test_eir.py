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

from oracle import ref
from paper_1304_2017_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_simulation_setup.json")


def gamma_pulse(L, dt, tau):
    """A causal low-pass response h(t) = t/tau^2 exp(-t/tau), sampled as
    h[m] = dt h(m dt); its transform 1/(1 + i 2 pi f tau)^2 has no zeros."""
    t = np.arange(L) * dt
    return dt * t / tau ** 2 * np.exp(-t / tau)


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
