"""Python binding of liboat (include/oat.h): argument marshalling only.

Every operator runs in the library's HIP kernels on the GPU; this module
never computes any part of H, H^T or FBP itself and has no CPU fallback.
torch is used for device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .synth import Geometry

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboat.so")

OAT_OK = 0
OAT_ERR_ARG = -1
OAT_ERR_GEOMETRY = -2
OAT_ERR_DTYPE = -3
OAT_ERR_DEVICE = -4
OAT_ERR_NOMEM = -5
OAT_ERR_INTERNAL = -6
OAT_F32 = 0
OAT_BF16 = 1
OAT_FLAG_SRT_ONLY = 1
OAT_FLAG_DETERMINISTIC = 2

EXPORTED = ("oat_plan_create", "oat_plan_create_ex", "oat_plan_destroy", "oat_project",
            "oat_backproject", "oat_fbp", "oat_last_error", "oat_plan_stats",
            "oat_plan_set_eir", "oat_deconvolve", "oat_sph_project", "oat_sph_backproject",
            "oat_sph_backproject_noalloc", "oat_plan_set_aperture",
            # include/oat_cnn.h
            "oat_conv3d_forward", "oat_conv3d_backward_weight_workspace",
            "oat_conv3d_backward_weight", "oat_adam_step", "oat_mse_workspace", "oat_mse")


class OatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oat status {code}: {msg}")
        self.code = code


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("z0", ctypes.c_double), ("n_det", ctypes.c_int32),
                ("det_xyz", ctypes.POINTER(ctypes.c_double)),
                ("det_area", ctypes.POINTER(ctypes.c_double)),
                ("n_t", ctypes.c_int32), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
                ("c0", ctypes.c_double), ("gamma", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("arc_table_bytes", ctypes.c_int64), ("segment_table_bytes", ctypes.c_int64)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load liboat.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; it must be loaded before this
        # library so both use the same one (loaded after, it finds no GPU).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(_LIB_PATH):
            raise ImportError(
                f"{_LIB_PATH} is missing: build it with `python -m paper_1304_2017_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        L.oat_plan_create.argtypes = [ctypes.POINTER(_Geom), ctypes.c_int, ctypes.POINTER(vp)]
        L.oat_plan_create.restype = ctypes.c_int
        L.oat_plan_create_ex.argtypes = [ctypes.POINTER(_Geom), ctypes.c_int,
                                         ctypes.POINTER(_Options), ctypes.POINTER(vp)]
        L.oat_plan_create_ex.restype = ctypes.c_int
        L.oat_plan_destroy.argtypes = [vp]
        L.oat_plan_destroy.restype = None
        for name in ("oat_project", "oat_backproject", "oat_fbp"):
            f = getattr(L, name)
            f.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_uint32, vp]
            f.restype = ctypes.c_int
        L.oat_plan_set_eir.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        L.oat_plan_set_eir.restype = ctypes.c_int
        L.oat_deconvolve.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_uint32, vp]
        L.oat_deconvolve.restype = ctypes.c_int
        d = ctypes.c_double
        L.oat_sph_project.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int, d, d,
                                      ctypes.c_uint32, vp]
        L.oat_sph_project.restype = ctypes.c_int
        L.oat_sph_backproject.argtypes = [vp, vp, ctypes.c_int, d, d, vp, ctypes.c_int,
                                          ctypes.c_uint32, vp]
        L.oat_sph_backproject.restype = ctypes.c_int
        L.oat_plan_set_aperture.argtypes = [vp, d, d, ctypes.c_int]
        L.oat_plan_set_aperture.restype = ctypes.c_int
        L.oat_sph_backproject_noalloc.argtypes = L.oat_sph_backproject.argtypes
        L.oat_sph_backproject_noalloc.restype = ctypes.c_int
        L.oat_last_error.argtypes = []
        L.oat_last_error.restype = ctypes.c_char_p
        L.oat_plan_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.oat_plan_stats.restype = ctypes.c_int
        ci, sz, i64, f = ctypes.c_int, ctypes.c_size_t, ctypes.c_int64, ctypes.c_float
        L.oat_conv3d_forward.argtypes = [vp, ci, ci, ci, ci, ci, vp, vp, ci, vp, ci, ci, vp, vp]
        L.oat_conv3d_forward.restype = ci
        L.oat_conv3d_backward_weight_workspace.argtypes = [ci, ci, ci, ci, ci]
        L.oat_conv3d_backward_weight_workspace.restype = sz
        L.oat_conv3d_backward_weight.argtypes = [vp, ci, vp, ci, ci, ci, ci, ci, ci, vp, vp, vp, sz,
                                                 vp]
        L.oat_conv3d_backward_weight.restype = ci
        L.oat_adam_step.argtypes = [vp, vp, vp, vp, i64, f, f, f, f, ci, vp]
        L.oat_adam_step.restype = ci
        L.oat_mse_workspace.argtypes = []
        L.oat_mse_workspace.restype = sz
        L.oat_mse.argtypes = [vp, ci, vp, ci, i64, vp, vp, vp, vp]
        L.oat_mse.restype = ci
        _lib = L
    return _lib


def last_error() -> str:
    return lib().oat_last_error().decode()


def _check(code: int):
    if code != OAT_OK:
        raise OatError(code, last_error())


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return OAT_F32
    if t.dtype == torch.bfloat16:
        return OAT_BF16
    raise TypeError(f"unsupported dtype {t.dtype}: use float32 or bfloat16")


class Plan:
    """Tables and workspace for one geometry on one device (oat_plan)."""

    def __init__(self, geom: Geometry, device: int = 0, arc_table="auto", segment_table="auto"):
        """arc_table, segment_table: "auto" (build it if it fits in 40% of
        free device memory), False / 0 (never), or a byte budget
        (oat_plan_options).  The plan tries the segment table first and
        builds the arc table only when it has none."""
        self.geom = geom
        self.device = int(device)
        self._eir = None
        self._xyz = np.ascontiguousarray(geom.det_xyz, dtype=np.float64).reshape(-1, 3)
        self._area = (None if geom.det_area is None
                      else np.ascontiguousarray(geom.det_area, dtype=np.float64))
        dp = ctypes.POINTER(ctypes.c_double)
        self._g = _Geom(geom.nx, geom.ny, geom.nz, geom.dx, geom.x0, geom.y0, geom.z0,
                        self._xyz.shape[0], self._xyz.ctypes.data_as(dp),
                        self._area.ctypes.data_as(dp) if self._area is not None else dp(),
                        geom.n_t, geom.dt, geom.t0, geom.c0, geom.gamma)
        def budget(v):
            if v == "auto" or v is None:
                return -1
            if v is False:
                return 0
            return int(v)

        self._opt = _Options(budget(arc_table), budget(segment_table))
        h = ctypes.c_void_p()
        _check(lib().oat_plan_create_ex(ctypes.byref(self._g), self.device,
                                        ctypes.byref(self._opt), ctypes.byref(h)))
        self._h = h

    # -- plumbing ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().oat_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        v = (ctypes.c_int64 * 13)()
        _check(lib().oat_plan_stats(self._h, v, 13))
        keys = ("rings", "bricks", "brick", "window", "workspace_bytes", "table_bytes",
                "arc_table_bytes", "arc_table_entries", "arc_table_build_us", "adj_calibration_us",
                "segment_table_bytes", "segment_table_entries", "segment_table_build_us")
        return dict(zip(keys, [int(x) for x in v]))

    def _prep(self, t, shape):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("expected a torch tensor on the GPU")
        if t.device.index != self.device:
            raise ValueError(f"tensor on cuda:{t.device.index}, plan on device {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return t

    def _stream(self, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    def _out(self, out, shape, dtype, like):
        import torch
        if out is None:
            out = torch.empty(shape, dtype=dtype or like.dtype, device=like.device)
        return self._prep(out, shape)

    @property
    def image_shape(self):
        return (self.geom.nz, self.geom.ny, self.geom.nx)

    @property
    def data_shape(self):
        return (self.geom.n_det, self.geom.n_t)

    # -- operators ----------------------------------------------------------
    def project(self, img, out=None, out_dtype=None, srt_only: bool = False, stream=None):
        """p = H img  (Eq. (dis_srt) then Eq. (dis_g2p)); srt_only gives g = G img."""
        img = self._prep(img, self.image_shape)
        out = self._out(out, self.data_shape, out_dtype, img)
        flags = OAT_FLAG_SRT_ONLY if srt_only else 0
        _check(lib().oat_project(self._h, ctypes.c_void_p(img.data_ptr()), _dtype_code(img),
                                 ctypes.c_void_p(out.data_ptr()), _dtype_code(out), flags,
                                 self._stream(stream)))
        return out

    def backproject(self, data, out=None, out_dtype=None, srt_only: bool = False, stream=None):
        """img = H^T data = G^T D^T data; srt_only gives G^T data."""
        data = self._prep(data, self.data_shape)
        out = self._out(out, self.image_shape, out_dtype, data)
        flags = OAT_FLAG_SRT_ONLY if srt_only else 0
        _check(lib().oat_backproject(self._h, ctypes.c_void_p(data.data_ptr()),
                                     _dtype_code(data), ctypes.c_void_p(out.data_ptr()),
                                     _dtype_code(out), flags, self._stream(stream)))
        return out

    def fbp(self, pres, out=None, out_dtype=None, stream=None):
        """Filtered backprojection of pressure data, Eq. (disfbp)."""
        pres = self._prep(pres, self.data_shape)
        out = self._out(out, self.image_shape, out_dtype, pres)
        _check(lib().oat_fbp(self._h, ctypes.c_void_p(pres.data_ptr()), _dtype_code(pres),
                             ctypes.c_void_p(out.data_ptr()), _dtype_code(out), 0,
                             self._stream(stream)))
        return out

    def set_eir(self, h):
        """Electrical impulse response h[m] = dt h^e(m dt) (Eq. (EIR)); None or
        an empty sequence removes it (oat_plan_set_eir; synchronous)."""
        taps = np.zeros(0) if h is None else np.ascontiguousarray(h, dtype=np.float64).ravel()
        _check(lib().oat_plan_set_eir(self._h, taps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      int(taps.size)))
        self._eir = taps.copy() if taps.size else None

    def sph_project(self, img, n_f: int, f_min: float, df: float, out=None, stream=None):
        """Spherical-voxel model, Eq. (dis_sph): complex64 [n_det][n_f]."""
        import torch
        img = self._prep(img, self.image_shape)
        if out is None:
            out = torch.empty((self.geom.n_det, n_f), device=img.device, dtype=torch.complex64)
        if out.dtype != torch.complex64:
            raise TypeError("sph_project output must be complex64")
        self._prep(out, (self.geom.n_det, n_f))
        _check(lib().oat_sph_project(self._h, ctypes.c_void_p(img.data_ptr()), _dtype_code(img),
                                     ctypes.c_void_p(out.data_ptr()), int(n_f), float(f_min),
                                     float(df), 0, self._stream(stream)))
        return out

    def sph_backproject(self, u, f_min: float, df: float, out=None, out_dtype=None, stream=None):
        """Eq. (sphbwd) (real part): u complex64 [n_det][n_f] -> image."""
        import torch
        if not isinstance(u, torch.Tensor) or u.dtype != torch.complex64 or u.dim() != 2:
            raise TypeError("sph_backproject expects complex64 data of shape [n_det, n_f]")
        n_f = int(u.shape[1])
        self._prep(u, (self.geom.n_det, n_f))
        if out is None:
            out = torch.empty(self.image_shape, device=u.device, dtype=out_dtype or torch.float32)
        self._prep(out, self.image_shape)
        _check(lib().oat_sph_backproject(self._h, ctypes.c_void_p(u.data_ptr()), n_f,
                                         float(f_min), float(df), ctypes.c_void_p(out.data_ptr()),
                                         _dtype_code(out), 0, self._stream(stream)))
        return out

    def set_aperture(self, width: float = 0.0, height: float = 0.0, m: int = 4):
        """Finite width x height (mm) transducer faces for the spherical-voxel
        model, m x m Gauss-Legendre nodes; (0, 0) restores point-like ones."""
        _check(lib().oat_plan_set_aperture(self._h, float(width), float(height), int(m)))

    def sph_backproject_noalloc(self, u, f_min: float, df: float, out, stream=None):
        """Eq. (sphbwd) into the caller's `out` through the entry point that
        allocates nothing (fixed per-GPU scratch; overlapping calls on one GPU
        race)."""
        import torch
        if not isinstance(u, torch.Tensor) or u.dtype != torch.complex64 or u.dim() != 2:
            raise TypeError("sph_backproject_noalloc expects complex64 data [n_det, n_f]")
        n_f = int(u.shape[1])
        self._prep(u, (self.geom.n_det, n_f))
        self._prep(out, self.image_shape)
        _check(lib().oat_sph_backproject_noalloc(
            self._h, ctypes.c_void_p(u.data_ptr()), n_f, float(f_min), float(df),
            ctypes.c_void_p(out.data_ptr()), _dtype_code(out), 0, self._stream(stream)))
        return out

    def deconvolve(self, u, f_cut: float, out=None, out_dtype=None, stream=None):
        """Hann-window Fourier deconvolution of the plan's EIR (Sec. IV.B),
        cutoff f_cut in cycles per time unit (MHz for microseconds)."""
        u = self._prep(u, self.data_shape)
        out = self._out(out, self.data_shape, out_dtype, u)
        _check(lib().oat_deconvolve(self._h, ctypes.c_void_p(u.data_ptr()), _dtype_code(u),
                                    ctypes.c_void_p(out.data_ptr()), _dtype_code(out),
                                    float(f_cut), 0, self._stream(stream)))
        return out
