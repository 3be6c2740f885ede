"""ctypes binding of the FP64 oracle (oat_ref.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.

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
        L.ref_count_points.argtypes = [G, _c_ip, ctypes.c_int]
        L.ref_count_points.restype = ctypes.c_long
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


def count_points(geom, rows=None):
    h = _GeomHolder(geom)
    rows, rp = _rows(h, rows)
    return int(lib().ref_count_points(h.ptr, rp, rows.size))


def max_threads():
    return int(lib().ref_max_threads())


def set_threads(n: int):
    """OpenMP threads of later calls (timing only)."""
    lib().ref_set_threads(int(n))
