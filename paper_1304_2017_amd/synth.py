"""Seeded synthetic inputs: measurement geometries, phantoms and data.

This module holds input generators only (transducer layouts, voxelised
phantoms, analytic pressure for uniform balls, noise).  It contains none of
the discrete operators (G, D, their adjoints, FBP); both the HIP path and the
FP64 oracle consume what it produces.

Geometry follows the paper's measurement set-up (Sec. III.A): transducers on
a sphere of radius R^s centred at the origin and a Cartesian grid of nodes
r_n = r_0 + dx*(ix, iy, iz).  The paper's own phantom and mouse data are not
available; seeded balls and ellipsoids of the same kind stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Geometry:
    """Problem statement of the imaging operators (lengths mm, times us)."""
    nx: int
    ny: int
    nz: int
    dx: float
    x0: float
    y0: float
    z0: float
    det_xyz: np.ndarray            # (Q, 3) float64
    n_t: int
    dt: float
    t0: float = 0.0
    c0: float = 1.5
    gamma: float = 1.0
    det_area: Optional[np.ndarray] = None   # (Q,) patch areas for FBP
    name: str = field(default="")

    @property
    def n_det(self) -> int:
        return int(self.det_xyz.shape[0])

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    def as_dict(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, dx=self.dx, x0=self.x0,
                    y0=self.y0, z0=self.z0, det_xyz=self.det_xyz,
                    det_area=self.det_area, n_t=self.n_t, dt=self.dt, t0=self.t0,
                    c0=self.c0, gamma=self.gamma)

    def node_coords(self):
        """Node coordinates as three broadcastable arrays (z, y, x order)."""
        z = self.z0 + self.dx * np.arange(self.nz)[:, None, None]
        y = self.y0 + self.dx * np.arange(self.ny)[None, :, None]
        x = self.x0 + self.dx * np.arange(self.nx)[None, None, :]
        return x, y, z

    def with_detectors(self, idx) -> "Geometry":
        """Same grid and sampling, keeping only the listed transducers."""
        idx = np.asarray(idx)
        area = None if self.det_area is None else self.det_area[idx]
        return Geometry(self.nx, self.ny, self.nz, self.dx, self.x0, self.y0, self.z0,
                        np.ascontiguousarray(self.det_xyz[idx]), self.n_t, self.dt,
                        self.t0, self.c0, self.gamma, area, self.name)


def centred_origin(n: int, dx: float) -> float:
    """x0 such that the n nodes are centred on 0."""
    return -0.5 * (n - 1) * dx


# ----------------------------------------------------------------------------
# Transducer layouts
# ----------------------------------------------------------------------------
def fibonacci_sphere(Q: int, Rs: float) -> np.ndarray:
    """Q points on the full sphere: z_i = 1-(2i+1)/Q, phi_i = i*pi*(3-sqrt5)."""
    i = np.arange(Q, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / Q
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([Rs * s * np.cos(phi), Rs * s * np.sin(phi), Rs * z], axis=1)


def fibonacci_hemisphere(Q: int, Rs: float) -> np.ndarray:
    """Q points on the lower hemisphere z < 0: z_i = -(i+1/2)/Q."""
    i = np.arange(Q, dtype=np.float64)
    z = -(i + 0.5) / Q
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([Rs * s * np.cos(phi), Rs * s * np.sin(phi), Rs * z], axis=1)


def ring_layout(n_rings: int, n_views: int, Rs: float, theta_min: float,
                dtheta: float):
    """Rings of constant polar angle theta = n_r*dtheta + theta_min with
    n_views transducers each at phi = 2*pi*n_v/n_views (Sec. III.A).
    Returns (positions (Q,3), patch areas Rs^2 dtheta dphi sin(theta))."""
    th = theta_min + dtheta * np.arange(n_rings)
    ph = 2.0 * math.pi * np.arange(n_views) / n_views
    T, P = np.meshgrid(th, ph, indexing="ij")
    xyz = np.stack([Rs * np.sin(T) * np.cos(P), Rs * np.sin(T) * np.sin(P),
                    Rs * np.cos(T)], axis=-1).reshape(-1, 3)
    area = (Rs * Rs * dtheta * (2.0 * math.pi / n_views) * np.sin(T)).reshape(-1)
    return xyz, area


# ----------------------------------------------------------------------------
# Phantoms (alpha_n = A(r_n), Eq. (coeffint): point samples at the nodes)
# ----------------------------------------------------------------------------
@dataclass
class Ball:
    centre: np.ndarray
    radius: float
    amplitude: float


def random_balls(rng: np.random.Generator, n: int, r_lo: float, r_hi: float,
                 fov_radius: float, a_lo: float = 0.5, a_hi: float = 1.0):
    """n balls, radius U(r_lo, r_hi), centre uniform in the ball of radius
    fov_radius - radius, amplitude U(a_lo, a_hi)."""
    balls = []
    for _ in range(n):
        r = rng.uniform(r_lo, r_hi)
        lim = max(fov_radius - r, 0.0)
        while True:
            c = rng.uniform(-lim, lim, size=3)
            if np.dot(c, c) <= lim * lim:
                break
        balls.append(Ball(c, r, rng.uniform(a_lo, a_hi)))
    return balls


def voxelise_balls(geom: Geometry, balls) -> np.ndarray:
    x, y, z = geom.node_coords()
    img = np.zeros(geom.shape)
    for b in balls:
        d2 = (x - b.centre[0]) ** 2 + (y - b.centre[1]) ** 2 + (z - b.centre[2]) ** 2
        img += np.where(d2 <= b.radius * b.radius, b.amplitude, 0.0)
    return img


@dataclass
class Ellipsoid:
    centre: np.ndarray
    semi_axes: np.ndarray
    rotation: np.ndarray    # 3x3, columns are the principal axes
    amplitude: float


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def random_ellipsoids(rng: np.random.Generator, n: int, geom: Geometry,
                      ax_lo: float, ax_hi: float, a_lo: float = 0.0,
                      a_hi: float = 1.0):
    """n ellipsoids: semi-axes U(ax_lo, ax_hi), uniformly random orientation
    (normalised Gaussian quaternion), centre uniform in the grid box shrunk by
    the largest semi-axis, amplitude U(a_lo, a_hi)."""
    lo = np.array([geom.x0, geom.y0, geom.z0])
    hi = lo + geom.dx * (np.array([geom.nx, geom.ny, geom.nz]) - 1)
    out = []
    for _ in range(n):
        ax = rng.uniform(ax_lo, ax_hi, size=3)
        m = ax.max()
        c = rng.uniform(lo + m, hi - m)
        out.append(Ellipsoid(c, ax, _random_rotation(rng), rng.uniform(a_lo, a_hi)))
    return out


def voxelise_ellipsoids(geom: Geometry, ells, dtype=np.float64) -> np.ndarray:
    """Additive point samples, evaluated slab by slab (bounded memory)."""
    img = np.zeros(geom.shape, dtype=dtype)
    xs = geom.x0 + geom.dx * np.arange(geom.nx)
    ys = geom.y0 + geom.dx * np.arange(geom.ny)
    zs = geom.z0 + geom.dx * np.arange(geom.nz)
    for e in ells:
        m = e.semi_axes.max()
        sl = []
        for coords, c in ((zs, e.centre[2]), (ys, e.centre[1]), (xs, e.centre[0])):
            i0 = int(np.searchsorted(coords, c - m, side="left"))
            i1 = int(np.searchsorted(coords, c + m, side="right"))
            sl.append(slice(i0, i1))
        Z = zs[sl[0]][:, None, None] - e.centre[2]
        Y = ys[sl[1]][None, :, None] - e.centre[1]
        X = xs[sl[2]][None, None, :] - e.centre[0]
        R = e.rotation
        u = (X * R[0, 0] + Y * R[1, 0] + Z * R[2, 0]) / e.semi_axes[0]
        v = (X * R[0, 1] + Y * R[1, 1] + Z * R[2, 1]) / e.semi_axes[1]
        w = (X * R[0, 2] + Y * R[1, 2] + Z * R[2, 2]) / e.semi_axes[2]
        inside = (u * u + v * v + w * w) <= 1.0
        img[sl[0], sl[1], sl[2]] += np.where(inside, e.amplitude, 0.0).astype(dtype)
    return img


def gaussian_blob(geom: Geometry, centre, sigma: float, amplitude: float = 1.0):
    x, y, z = geom.node_coords()
    d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return amplitude * np.exp(-d2 / (2.0 * sigma * sigma))


# ----------------------------------------------------------------------------
# Analytic pressure of uniform balls (continuous model, Eqs. (srt), (g2p))
# ----------------------------------------------------------------------------
def nwave_balls(geom: Geometry, balls) -> np.ndarray:
    """Pressure p(r_q, t_k) of a sum of uniform balls for point transducers.

    For a ball of amplitude A, radius a at distance d from the transducer the
    spherical Radon transform is g = A*pi*rho*(a^2-(d-rho)^2)/d for
    |d-rho| <= a (rho = c0 t), and p = Gamma/(4 pi c0^2) d/dt (g/t) gives
    p = (A Gamma / 2) (d - c0 t) / d inside that window, 0 outside.
    """
    t = geom.t0 + geom.dt * np.arange(geom.n_t)
    rho = geom.c0 * t
    out = np.zeros((geom.n_det, geom.n_t))
    for b in balls:
        d = np.linalg.norm(geom.det_xyz - b.centre[None, :], axis=1)[:, None]
        inside = np.abs(rho[None, :] - d) <= b.radius
        out += np.where(inside, 0.5 * b.amplitude * geom.gamma * (d - rho[None, :]) / d, 0.0)
    return out


def blur_time(geom: Geometry, data: np.ndarray, fwhm: float) -> np.ndarray:
    """Each transducer's samples convolved with a Gaussian of the given FWHM
    (time units), sampled on the data grid and normalised to unit sum, zero
    beyond the record (the simulation data of Sec. IV.A: the N-wave of
    uniform spheres blurred in time like the phantom in space)."""
    from scipy.ndimage import gaussian_filter1d
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0))) / geom.dt
    return gaussian_filter1d(np.asarray(data, dtype=np.float64), sigma, axis=1, mode="constant",
                             truncate=6.0)


def gaussian_noise(rng: np.random.Generator, data: np.ndarray, rel: float) -> np.ndarray:
    """Additive white noise with sigma = rel * max|data|."""
    return data + rng.normal(scale=rel * float(np.max(np.abs(data))), size=data.shape)


# ----------------------------------------------------------------------------
# The workloads used by the tests and the benchmark
# ----------------------------------------------------------------------------
def config_small(seed: int = 0):
    """32^3 nodes at 0.5 mm with 3 seeded uniform balls (radii 1-4 mm,
    amplitudes U(0.5,1)); 64 transducers at Fibonacci points on a sphere of
    radius 25 mm; 256 samples at 10 MHz; c0 = 1.5 mm/us."""
    n, dx = 32, 0.5
    o = centred_origin(n, dx)
    geom = Geometry(n, n, n, dx, o, o, o, fibonacci_sphere(64, 25.0), 256, 0.1,
                    0.0, 1.5, 1.0, name="32^3 / 64 transducers / 256 samples")
    rng = np.random.default_rng(seed)
    balls = random_balls(rng, 3, 1.0, 4.0, 7.0)
    return geom, balls, voxelise_balls(geom, balls)


def config_large_geometry():
    """256^3 nodes at 0.1 mm; 2048 transducers at Fibonacci points on the
    lower hemisphere of radius 40 mm (patch area 2 pi Rs^2 / Q); 1024 samples
    at 20 MHz; c0 = 1.5 mm/us."""
    n, dx = 256, 0.1
    o = centred_origin(n, dx)
    Q, Rs = 2048, 40.0
    return Geometry(n, n, n, dx, o, o, o, fibonacci_hemisphere(Q, Rs), 1024, 0.05,
                    0.0, 1.5, 1.0, np.full(Q, 2.0 * math.pi * Rs * Rs / Q),
                    name="256^3 / 2048 transducers / 1024 samples")


def config_large(seed: int = 0, dtype=np.float32):
    """config_large_geometry with 40 seeded ellipsoids (semi-axes
    0.3-3 mm, amplitudes U(0,1))."""
    geom = config_large_geometry()
    rng = np.random.default_rng(seed)
    ells = random_ellipsoids(rng, 40, geom, 0.3, 3.0, 0.0, 1.0)
    return geom, ells, voxelise_ellipsoids(geom, ells, dtype=dtype)


def config_sph(seed: int = 0, dtype=np.float32, n: int = 64):
    """The spherical-voxel model's workload: the 25.6 mm field of view and
    2048-transducer hemisphere of config_large_geometry at n^3 nodes
    (0.4 mm voxels at the default 64^3), 40 seeded ellipsoids as in
    config_large.  (The dense frequency-domain sum costs
    n_det x n_f x voxels terms, so the voxel count is kept moderate.)"""
    dx = 25.6 / n
    o = centred_origin(n, dx)
    Q, Rs = 2048, 40.0
    geom = Geometry(n, n, n, dx, o, o, o, fibonacci_hemisphere(Q, Rs), 1024, 0.05, 0.0, 1.5, 1.0,
                    np.full(Q, 2.0 * math.pi * Rs * Rs / Q),
                    name=f"{n}^3 / 2048 transducers (spherical voxels)")
    rng = np.random.default_rng(seed)
    ells = random_ellipsoids(rng, 40, geom, 0.3, 3.0, 0.0, 1.0)
    return geom, voxelise_ellipsoids(geom, ells, dtype=dtype)


def blurred_ball(geom: Geometry, ball: Ball, sigma: float) -> np.ndarray:
    """A uniform ball convolved with an isotropic Gaussian of standard
    deviation sigma, sampled at the nodes: with r the distance to the centre,
    A { [erf((a-r)/(s sqrt2)) + erf((a+r)/(s sqrt2))]/2
        + s/(r sqrt(2 pi)) [exp(-(a+r)^2/(2 s^2)) - exp(-(a-r)^2/(2 s^2))] }."""
    from scipy.special import erf
    X, Y, Z = geom.node_coords()
    r = np.sqrt((X - ball.centre[0]) ** 2 + (Y - ball.centre[1]) ** 2 + (Z - ball.centre[2]) ** 2)
    a, s = ball.radius, sigma
    rs = np.maximum(r, 1e-9)
    v = 0.5 * (erf((a - r) / (s * math.sqrt(2.0))) + erf((a + r) / (s * math.sqrt(2.0))))
    v += s / (rs * math.sqrt(2.0 * math.pi)) * (np.exp(-(a + r) ** 2 / (2 * s * s)) -
                                                  np.exp(-(a - r) ** 2 / (2 * s * s)))
    return ball.amplitude * v


def config_c_geometry():
    """192^3 nodes at 0.1 mm; 4096 transducers on a full Fibonacci sphere of
    radius 40 mm; 1024 samples at 20 MHz (the PLS workload)."""
    n, dx = 192, 0.1
    o = centred_origin(n, dx)
    return Geometry(n, n, n, dx, o, o, o, fibonacci_sphere(4096, 40.0), 1024, 0.05, 0.0, 1.5, 1.0,
                    name="192^3 / 4096 transducers / 1024 samples")


def config_c(seed: int = 0):
    """config_c_geometry with data = analytic N-wave of 9 seeded uniform balls
    (radii 0.5-2 mm in the central 8 mm) plus white noise of 2% of max|u|."""
    geom = config_c_geometry()
    rng = np.random.default_rng(seed)
    balls = random_balls(rng, 9, 0.5, 2.0, 8.0)
    u = gaussian_noise(rng, nwave_balls(geom, balls), 0.02)
    return geom, balls, u


def config_e_geometry():
    """256^3 nodes at 0.1 mm; 8192 transducers on a full Fibonacci sphere of
    radius 45 mm; 1024 samples at 20 MHz."""
    n, dx = 256, 0.1
    o = centred_origin(n, dx)
    return Geometry(n, n, n, dx, o, o, o, fibonacci_sphere(8192, 45.0), 1024, 0.05, 0.0, 1.5, 1.0,
                    name="256^3 / 8192 transducers / 1024 samples")


def config_e(seed: int = 0, dtype=np.float32):
    """config_e_geometry with 60 seeded ellipsoids as in config_large."""
    geom = config_e_geometry()
    rng = np.random.default_rng(seed)
    ells = random_ellipsoids(rng, 60, geom, 0.3, 3.0, 0.0, 1.0)
    return geom, ells, voxelise_ellipsoids(geom, ells, dtype=dtype)


def config_p_geometry():
    """The paper's simulation shape: 210 x 210 x 440 nodes at 0.14 mm; 64 rings
    x 90 views on a sphere of radius 65 mm at theta_n = (n + 1/2) pi/64, patch
    areas Rs^2 (pi/64)(2 pi/90) sin(theta); 1022 samples at 20 MHz from
    t0 = 17.5 us; c0 = 1.54 mm/us."""
    nx, ny, nz, dx = 210, 210, 440, 0.14
    xyz, area = ring_layout(64, 90, 65.0, math.pi / 128.0, math.pi / 64.0)
    return Geometry(nx, ny, nz, dx, centred_origin(nx, dx), centred_origin(ny, dx),
                    centred_origin(nz, dx), xyz, 1022, 0.05, 17.5, 1.54, 1.0, area,
                    name="210x210x440 / 64x90 ring views / 1022 samples")


def config_p_rings(n_rings: int, n_views: int):
    """config_p_geometry with n_rings x n_views ring views: rings at
    theta_n = (n + 1/2) pi / n_rings (full polar range, the paper's
    theta_min = pi/256 at 128 rings) and n_views views over 2 pi."""
    g = config_p_geometry()
    xyz, area = ring_layout(n_rings, n_views, 65.0, math.pi / (2 * n_rings), math.pi / n_rings)
    return Geometry(g.nx, g.ny, g.nz, g.dx, g.x0, g.y0, g.z0, xyz, g.n_t, g.dt, g.t0, g.c0, g.gamma,
                    area, name=f"210x210x440 / {n_rings}x{n_views} ring views / 1022 samples")


def config_p_data(geom: Geometry, balls) -> np.ndarray:
    """The paper's simulated pressure for config_p's balls on `geom`: the
    N-wave of the uniform balls blurred in time by a Gaussian of FWHM
    0.5 us (0.77 mm at c0 = 1.54 mm/us, the phantom's blur)."""
    return blur_time(geom, nwave_balls(geom, balls), 0.5)


def config_p(seed: int = 0, dtype=np.float32):
    """config_p_geometry with 9 seeded uniform balls (radii 1-4 mm, inside the
    central 12 mm) blurred by a Gaussian of FWHM 0.77 mm."""
    geom = config_p_geometry()
    rng = np.random.default_rng(seed)
    balls = random_balls(rng, 9, 1.0, 4.0, 12.0)
    sigma = 0.77 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    img = np.zeros(geom.shape)
    for b in balls:
        img += blurred_ball(geom, b, sigma)
    return geom, balls, img.astype(dtype)


def config_d_geometry():
    """128^3 nodes at 0.1 mm; 1024 transducers on a full Fibonacci sphere of
    radius 25 mm; 512 samples at 20 MHz (the training workload)."""
    n, dx = 128, 0.1
    o = centred_origin(n, dx)
    return Geometry(n, n, n, dx, o, o, o, fibonacci_sphere(1024, 25.0), 512, 0.05, 0.0, 1.5, 1.0,
                    name="128^3 / 1024 transducers / 512 samples")


def config_d_phantoms(count: int = 64, seed: int = 0, dtype=np.float32):
    """`count` seeded phantoms on config_d_geometry, each 15-60 ellipsoids as
    in config_large."""
    geom = config_d_geometry()
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        ells = random_ellipsoids(rng, int(rng.integers(15, 61)), geom, 0.3, 3.0, 0.0, 1.0)
        out.append(voxelise_ellipsoids(geom, ells, dtype=dtype))
    return geom, out


def gamma_pulse(taps: int, dt: float, tau: float) -> np.ndarray:
    """A synthetic transducer electrical impulse response for Eq. (EIR):
    h[m] = dt h(m dt) with the causal low-pass pulse h(t) = t/tau^2 exp(-t/tau)
    (unit area; its transform 1/(1 + i 2 pi f tau)^2 has no zeros).  The
    paper's measured EIR is not available; this stands in for it."""
    t = np.arange(taps) * dt
    return dt * t / tau ** 2 * np.exp(-t / tau)

