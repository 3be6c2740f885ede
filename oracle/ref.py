"""ctypes binding of the FP64 oracle (oat_ref.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.

The transducer-response functions at the end (eir, eir_adj, deconvolve) are
plain numpy.

All arrays are numpy float64, C-contiguous.  Geometry is passed as a dict
with keys nx, ny, nz, dx, x0, y0, z0, det_xyz (Q x 3), det_area (Q or None),
n_t, dt, t0, c0, gamma.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int)
_c_lp = ctypes.POINTER(ctypes.c_long)


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("nq", ctypes.c_int), ("rq", _c_dp), ("aq", _c_dp),
                ("nt", ctypes.c_int), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
                ("c0", ctypes.c_double), ("gamma", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        L = ctypes.CDLL(path)
        G = ctypes.POINTER(_Geom)
        L.ref_support_radius.argtypes = [G]
        L.ref_support_radius.restype = ctypes.c_double
        L.ref_srt_rows.argtypes = [G, _c_dp, _c_ip, ctypes.c_int, _c_dp]
        L.ref_srt_adj_rows.argtypes = [G, _c_dp, _c_ip, ctypes.c_int, _c_dp]
        L.ref_diff.argtypes = [G, ctypes.c_int, _c_dp, _c_dp]
        L.ref_diff_adj.argtypes = [G, ctypes.c_int, _c_dp, _c_dp]
        L.ref_project_rows.argtypes = [G, _c_dp, _c_ip, ctypes.c_int, _c_dp]
        L.ref_backproject_rows.argtypes = [G, _c_dp, _c_ip, ctypes.c_int, _c_dp]
        L.ref_fbp_voxels.argtypes = [G, _c_dp, _c_lp, ctypes.c_long, _c_dp]
        L.ref_shell_points.argtypes = [G, ctypes.c_int, ctypes.c_int, _c_dp, ctypes.c_long]
        L.ref_shell_points.restype = ctypes.c_long
        L.ref_max_threads.restype = ctypes.c_int
        L.ref_set_threads.argtypes = [ctypes.c_int]
        L.ref_set_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_c_dp)


class _GeomHolder:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, geom):
        self.rq = np.ascontiguousarray(geom["det_xyz"], dtype=np.float64).reshape(-1, 3)
        area = geom.get("det_area")
        self.aq = None if area is None else np.ascontiguousarray(area, dtype=np.float64)
        self.s = _Geom(int(geom["nx"]), int(geom["ny"]), int(geom["nz"]),
                       float(geom["dx"]), float(geom["x0"]), float(geom["y0"]),
                       float(geom["z0"]), int(self.rq.shape[0]), _dp(self.rq),
                       _dp(self.aq) if self.aq is not None else _c_dp(),
                       int(geom["n_t"]), float(geom["dt"]), float(geom["t0"]),
                       float(geom["c0"]), float(geom["gamma"]))
        self.nq = self.rq.shape[0]
        self.K = int(geom["n_t"])
        self.shape = (int(geom["nz"]), int(geom["ny"]), int(geom["nx"]))

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def _rows(h, rows):
    if rows is None:
        rows = np.arange(h.nq, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    return rows, rows.ctypes.data_as(_c_ip)


def support_radius(geom):
    h = _GeomHolder(geom)
    return lib().ref_support_radius(h.ptr)


def srt(geom, alpha, rows=None):
    """G alpha for the listed transducer rows -> (len(rows), K)."""
    h = _GeomHolder(geom)
    a = np.ascontiguousarray(alpha, dtype=np.float64).reshape(h.shape)
    rows, rp = _rows(h, rows)
    g = np.zeros((rows.size, h.K))
    lib().ref_srt_rows(h.ptr, _dp(a), rp, rows.size, _dp(g))
    return g


def srt_adj(geom, gp, rows=None):
    """G^T applied to data given for the listed rows -> image (nz, ny, nx)."""
    h = _GeomHolder(geom)
    rows, rp = _rows(h, rows)
    d = np.ascontiguousarray(gp, dtype=np.float64).reshape(rows.size, h.K)
    out = np.zeros(h.shape)
    lib().ref_srt_adj_rows(h.ptr, _dp(d), rp, rows.size, _dp(out))
    return out


def diff(geom, g):
    h = _GeomHolder(geom)
    g = np.ascontiguousarray(g, dtype=np.float64)
    g2 = g.reshape(-1, h.K)
    p = np.zeros_like(g2)
    lib().ref_diff(h.ptr, g2.shape[0], _dp(g2), _dp(p))
    return p.reshape(g.shape)


def diff_adj(geom, y):
    h = _GeomHolder(geom)
    y = np.ascontiguousarray(y, dtype=np.float64)
    y2 = y.reshape(-1, h.K)
    gp = np.zeros_like(y2)
    lib().ref_diff_adj(h.ptr, y2.shape[0], _dp(y2), _dp(gp))
    return gp.reshape(y.shape)


def project(geom, alpha, rows=None):
    """H alpha = D G alpha for the listed rows -> (len(rows), K)."""
    h = _GeomHolder(geom)
    a = np.ascontiguousarray(alpha, dtype=np.float64).reshape(h.shape)
    rows, rp = _rows(h, rows)
    p = np.zeros((rows.size, h.K))
    lib().ref_project_rows(h.ptr, _dp(a), rp, rows.size, _dp(p))
    return p


def backproject(geom, y, rows=None):
    """H^T y = G^T D^T y using the listed rows of y -> image."""
    h = _GeomHolder(geom)
    rows, rp = _rows(h, rows)
    d = np.ascontiguousarray(y, dtype=np.float64).reshape(rows.size, h.K)
    out = np.zeros(h.shape)
    lib().ref_backproject_rows(h.ptr, _dp(d), rp, rows.size, _dp(out))
    return out


def fbp(geom, p, voxels=None):
    """Eq. (disfbp).  voxels: flat indices to evaluate (None = whole image)."""
    h = _GeomHolder(geom)
    p = np.ascontiguousarray(p, dtype=np.float64).reshape(h.nq, h.K)
    if voxels is None:
        out = np.zeros(h.shape)
        lib().ref_fbp_voxels(h.ptr, _dp(p), _c_lp(), 0, _dp(out))
        return out
    vs = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.zeros(vs.size)
    lib().ref_fbp_voxels(h.ptr, _dp(p), vs.ctypes.data_as(_c_lp), vs.size, _dp(out))
    return out


def shell_points(geom, q, k):
    """The quadrature points of shell (q, k) that G and G^T visit, as an
    (n, 4) array of rows (x, y, z, weight), in visiting order."""
    h = _GeomHolder(geom)
    n = int(lib().ref_shell_points(h.ptr, int(q), int(k), _c_dp(), 0))
    out = np.zeros((max(n, 1), 4))
    lib().ref_shell_points(h.ptr, int(q), int(k), _dp(out), n)
    return out[:n]


def max_threads():
    return int(lib().ref_max_threads())


def set_threads(n: int):
    """OpenMP threads of later calls (timing only)."""
    lib().ref_set_threads(int(n))


# ---------------------------------------------------------------------------
# Transducer electrical impulse response (EIR), plain numpy in FP64.
# ---------------------------------------------------------------------------
def eir_matrix(h, K):
    """K x K matrix of Eq. (EIR): M[k, kappa] = h[k - 1 - kappa], with
    h[m] = 0 outside [0, len(h)).  (The printed index k - 1 - kappa delays the
    response by one sample; taken as printed.)"""
    h = np.asarray(h, dtype=np.float64)
    k = np.arange(K)[:, None]
    kappa = np.arange(K)[None, :]
    m = k - 1 - kappa
    inside = (m >= 0) & (m < h.size)
    return np.where(inside, h[np.clip(m, 0, h.size - 1)], 0.0)


def eir(h, p):
    """H^e p, Eq. (EIR), applied to every row of p [Q][K]."""
    p = np.asarray(p, dtype=np.float64)
    return p @ eir_matrix(h, p.shape[-1]).T


def eir_adj(h, u):
    """H^e^T u from the adjoint formula of Sec. II.B.3:
    p'[k] = sum_kappa h[kappa - 1 - k] u[kappa], for every row of u."""
    h = np.asarray(h, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    K = u.shape[-1]
    k = np.arange(K)[:, None]
    kappa = np.arange(K)[None, :]
    m = kappa - 1 - k
    inside = (m >= 0) & (m < h.size)
    A = np.where(inside, h[np.clip(m, 0, h.size - 1)], 0.0)   # A[k, kappa]
    return u @ A.T


def hann(f, fc):
    """Hann window of the deconvolution (Sec. IV.B, experimental data):
    W(f) = (1 - cos(pi (fc - |f|) / fc)) / 2 for |f| <= fc, 0 beyond."""
    af = np.abs(np.asarray(f, dtype=np.float64))
    return np.where(af <= fc, 0.5 * (1.0 - np.cos(np.pi * (fc - af) / fc)), 0.0)


def deconv_length(K):
    """FFT length of the deconvolution: the power of two >= 2K, so the
    division undoes the linear (not circular) convolution of a K-sample
    record."""
    n = 1
    while n < 2 * K:
        n *= 2
    return n


def deconvolve(h, u, dt, fc):
    """Fourier deconvolution with a Hann window (Sec. IV.B): per row of u,
    p~(f) = u~(f) W(f) / h~(f), h~ the transform of Eq. (EIR)'s response
    (one-sample delay included); bins with h~ = 0 give 0.  Rows are zero-padded
    to deconv_length(K); the first K samples of the inverse are returned."""
    u = np.asarray(u, dtype=np.float64)
    K = u.shape[-1]
    N = deconv_length(K)
    hd = np.zeros(N)
    hd[1:1 + len(h)] = h
    Ht = np.fft.fft(hd)
    W = hann(np.fft.fftfreq(N, d=dt), fc)
    Ut = np.fft.fft(u, n=N, axis=-1)
    nz = Ht != 0
    filt = np.zeros(N, dtype=np.complex128)
    filt[nz] = W[nz] / Ht[nz]
    return np.fft.ifft(Ut * filt, axis=-1).real[..., :K]


def project_eir(geom, h, alpha, rows=None):
    """H^e D G alpha (Eq. (EIR) after Eq. (dis_g2p)), the listed rows."""
    return eir(h, project(geom, alpha, rows=rows))


def backproject_eir(geom, h, y, rows=None):
    """G^T D^T H^e^T y using the listed rows of y."""
    return backproject(geom, eir_adj(h, y), rows=rows)


# ---------------------------------------------------------------------------
# Spherical-voxel imaging model (Sec. II.B.2), point-like transducers, plain
# numpy in FP64.
# ---------------------------------------------------------------------------
def sph_freqs(n_f, f_min, df):
    """Frequency samples f_l = f_min + l df, l = 0 .. n_f - 1 (the listings'
    form; Eq. (dis_sph) is the case f_min = 0)."""
    return f_min + df * np.arange(n_f, dtype=np.float64)


def sph_p0(f, geom):
    """Eq. (p0f) with beta c0^3 / Cp = Gamma c0 and an ideal EIR (h^e = 1):
    p0(f) = -j Gamma c0 / f [ dx/(2 c0) cos(pi f dx / c0) - sin(pi f dx / c0) / (2 pi f) ],
    0 at f = 0 (its limit)."""
    f = np.asarray(f, dtype=np.float64)
    c0, dx, gam = geom["c0"], geom["dx"], geom["gamma"]
    out = np.zeros(f.shape, dtype=np.complex128)
    nz = f != 0
    fn = f[nz]
    br = dx / (2 * c0) * np.cos(np.pi * fn * dx / c0) - np.sin(np.pi * fn * dx / c0) / (2 * np.pi * fn)
    out[nz] = -1j * gam * c0 / fn * br
    return out


def _nodes(geom):
    nx, ny, nz = geom["nx"], geom["ny"], geom["nz"]
    dx = geom["dx"]
    z, y, x = np.meshgrid(geom["z0"] + dx * np.arange(nz), geom["y0"] + dx * np.arange(ny),
                          geom["x0"] + dx * np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)   # [N][3], flat index of [nz][ny][nx]


def sph_face_points(geom, q, aperture):
    """Quadrature of (1/S_q) times the surface integral over the face S_q in
    the SIR of Eq. (dis_sph): (points [S][3], weights [S] summing to 1).

    aperture None: point-like transducers, the single point r_q.  Else
    (width, height, m): the face is the flat width x height rectangle (mm)
    centred at r_q and normal to r_q, its width along the unit polar vector
    e1 = (cos t cos p, cos t sin p, -sin t) and its height along
    e2 = (sin p, -cos p, 0) of r_q = |r_q| (sin t cos p, sin t sin p, cos t),
    sampled by the m x m Gauss-Legendre product rule (numpy's nodes and
    weights on [-1, 1], scaled to the face)."""
    rq = np.asarray(geom["det_xyz"], dtype=np.float64).reshape(-1, 3)[q]
    if aperture is None:
        return rq[None, :], np.ones(1)
    w, h, m = aperture
    dist = float(np.linalg.norm(rq))
    t = np.arccos(rq[2] / dist)
    p = np.arctan2(rq[1], rq[0])
    e1 = np.array([np.cos(t) * np.cos(p), np.cos(t) * np.sin(p), -np.sin(t)])
    e2 = np.array([np.sin(p), -np.cos(p), 0.0])
    x, wx = np.polynomial.legendre.leggauss(int(m))
    pts, wts = [], []
    for i in range(int(m)):
        for j in range(int(m)):
            pts.append(rq + 0.5 * w * x[i] * e1 + 0.5 * h * x[j] * e2)
            wts.append(0.25 * wx[i] * wx[j])
    return np.array(pts), np.array(wts)


def sph_sir(geom, q, r, f, aperture=None):
    """(1/S_q) h~_q(r, f) of Eq. (dis_sph) for points r [N][3] and frequencies
    f [L]: the face average of exp(-j 2 pi f |r^s - r| / c0) / (2 pi |r^s - r|)
    by sph_face_points' rule -> [L][N] complex."""
    pts, wts = sph_face_points(geom, q, aperture)
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros((f.size, r.shape[0]), dtype=np.complex128)
    for ps, ws in zip(pts, wts):
        d = np.linalg.norm(r - ps, axis=1)
        out += ws * np.exp(-2j * np.pi * np.outer(f, d) / geom["c0"]) / (2 * np.pi * d)
    return out


def sph_project(geom, alpha, n_f, f_min, df, rows=None, aperture=None):
    """Eq. (dis_sph): u[q, l] = p0(f_l) sum_n alpha_n (1/S_q) h~_q(r_n, f_l)
    (sph_sir; point-like transducers for aperture None: exp(-j 2 pi f_l
    d_qn / c0) / (2 pi d_qn), d_qn = |r_q - r_n|).  alpha [nz][ny][nx] real
    -> u [Q][n_f] complex, or the listed rows only."""
    r = _nodes(geom)
    a = np.asarray(alpha, dtype=np.float64).ravel()
    f = sph_freqs(n_f, f_min, df)
    p0 = sph_p0(f, geom)
    rq = np.asarray(geom["det_xyz"], dtype=np.float64).reshape(-1, 3)
    qs = np.arange(rq.shape[0]) if rows is None else np.asarray(rows)
    u = np.zeros((qs.size, n_f), dtype=np.complex128)
    for i, q in enumerate(qs):
        u[i] = p0 * (sph_sir(geom, q, r, f, aperture) @ a)
    return u


def sph_backproject(geom, u, n_f, f_min, df, voxels=None, aperture=None):
    """Eq. (sphbwd): [H^T u]_n = sum_{q,l} u[q,l] conj(p0(f_l)) conj((1/S_q) h~_q(r_n, f_l)).
    Returns its real part [nz][ny][nx] (the image is real, so this is the
    adjoint of sph_project over real images), or at the listed flat voxel
    indices."""
    r = _nodes(geom)
    if voxels is not None:
        r = r[np.asarray(voxels)]
    f = sph_freqs(n_f, f_min, df)
    p0c = np.conj(sph_p0(f, geom))
    rq = np.asarray(geom["det_xyz"], dtype=np.float64).reshape(-1, 3)
    u = np.asarray(u, dtype=np.complex128).reshape(rq.shape[0], n_f)
    out = np.zeros(r.shape[0], dtype=np.complex128)
    for q in range(rq.shape[0]):
        out += (u[q] * p0c) @ np.conj(sph_sir(geom, q, r, f, aperture))
    if voxels is not None:
        return out.real
    return out.real.reshape(geom["nz"], geom["ny"], geom["nx"])
