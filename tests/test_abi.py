"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/oat.h declares, and rejects bad arguments on the host before
touching a device.  Also runs the host check of the ring/brick arc geometry
used by the G kernels."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1304_2017_amd import oat, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(oat_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = oat.lib()
    names = _declared()
    assert set(names) == set(oat.EXPORTED)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", oat.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (oat_\w+)", out))
    assert set(names) <= exported


def _geom(**kw):
    g, _, _ = synth.config_small(0)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def _create(geom):
    p = oat._Geom()
    xyz = np.ascontiguousarray(geom.det_xyz, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    p = oat._Geom(geom.nx, geom.ny, geom.nz, geom.dx, geom.x0, geom.y0, geom.z0,
                  xyz.shape[0], xyz.ctypes.data_as(dp), dp(), geom.n_t, geom.dt, geom.t0,
                  geom.c0, geom.gamma)
    h = ctypes.c_void_p()
    rc = oat.lib().oat_plan_create(ctypes.byref(p), 0, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(det_xyz=np.array([[5.0, 0.0, 0.0]])),    # transducer inside the support sphere
    dict(dx=0.0), dict(dx=-1.0), dict(n_t=2), dict(n_t=5000), dict(dt=0.0),
    dict(c0=0.0), dict(gamma=0.0), dict(nx=0), dict(dx=float("nan")),
])
def test_invalid_geometry_is_rejected_before_launch(kw):
    rc, h = _create(_geom(**kw))
    assert rc == oat.OAT_ERR_GEOMETRY
    assert not h.value
    assert oat.last_error() != ""


def test_negative_table_budget_is_rejected():
    g = _geom()
    xyz = np.ascontiguousarray(g.det_xyz, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    p = oat._Geom(g.nx, g.ny, g.nz, g.dx, g.x0, g.y0, g.z0, xyz.shape[0], xyz.ctypes.data_as(dp),
                  dp(), g.n_t, g.dt, g.t0, g.c0, g.gamma)
    h = ctypes.c_void_p()
    opt = oat._Options(-2, -1)
    assert oat.lib().oat_plan_create_ex(ctypes.byref(p), 0, ctypes.byref(opt),
                                        ctypes.byref(h)) == oat.OAT_ERR_ARG
    assert not h.value and "arc_table_bytes" in oat.last_error()
    opt = oat._Options(-1, -3)
    assert oat.lib().oat_plan_create_ex(ctypes.byref(p), 0, ctypes.byref(opt),
                                        ctypes.byref(h)) == oat.OAT_ERR_ARG
    assert not h.value and "segment_table_bytes" in oat.last_error()


def test_null_arguments():
    L = oat.lib()
    assert L.oat_plan_create(None, 0, None) == oat.OAT_ERR_ARG
    assert L.oat_plan_create_ex(None, 0, None, None) == oat.OAT_ERR_ARG
    assert L.oat_project(None, None, 0, None, 0, 0, None) == oat.OAT_ERR_ARG
    assert L.oat_backproject(None, None, 0, None, 0, 0, None) == oat.OAT_ERR_ARG
    assert L.oat_fbp(None, None, 0, None, 0, 0, None) == oat.OAT_ERR_ARG
    assert L.oat_sph_backproject_noalloc(None, None, 16, 0.0, 0.1, None, 0, 0,
                                         None) == oat.OAT_ERR_ARG
    assert "null" in oat.last_error()
    L.oat_plan_destroy(None)


def test_host_arc_geometry_is_a_superset(tmp_path):
    exe = tmp_path / "arc_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_1304_2017_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "arc_check.cpp"), "-o", str(exe)],
                   check=True)
    for seed in (3, 4):
        r = subprocess.run([str(exe), "600", str(seed)], capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.startswith("OK"), r.stdout
        rings, inside = map(int, r.stdout.split()[1:3])
        assert inside > 10000


def test_host_fbp_floor_thresholds(tmp_path):
    exe = tmp_path / "fbp_floor_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_1304_2017_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "fbp_floor_check.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK"), r.stdout
    assert int(r.stdout.split()[1]) > 1000000


def test_flag_and_status_constants_match_the_header():
    """The binding's flag, dtype and status constants equal the header's."""
    text = open(os.path.join(ROOT, "include", "oat.h")).read()
    defines = {m.group(1): int(m.group(2)) for m in
               re.finditer(r"#define\s+(OAT_FLAG_\w+)\s+(\d+)u", text)}
    assert defines == {"OAT_FLAG_SRT_ONLY": oat.OAT_FLAG_SRT_ONLY,
                       "OAT_FLAG_DETERMINISTIC": oat.OAT_FLAG_DETERMINISTIC}
    enums = {m.group(1): int(m.group(2)) for m in
             re.finditer(r"\b(OAT_(?:OK|ERR_\w+|F32|BF16))\s*=\s*(-?\d+)", text)}
    for name, value in enums.items():
        assert getattr(oat, name) == value, name
    assert {"OAT_OK", "OAT_ERR_ARG", "OAT_ERR_GEOMETRY", "OAT_F32", "OAT_BF16"} <= set(enums)


def _fbp_window_workloads():
    """Every workload geometry: the 32^3, 256^3 (2048 hemisphere and 8192
    sphere), 192^3, 128^3 and paper-shape cases, and grids with ragged,
    off-centre and t0 != 0 timing."""
    from paper_1304_2017_amd import synth
    g = [synth.config_small(0)[0], synth.config_large_geometry(), synth.config_c_geometry(),
         synth.config_d_geometry(), synth.config_e_geometry(), synth.config_p_geometry()]
    for n, dx, off, Q, Rs, K, dt, t0 in [((37, 29, 23), 0.45, (0.3, -0.7, 0.2), 24, 21.0, 300, 0.08, 0.0),
                                         ((41, 22, 3), 0.3, (-1.0, 0.5, 0.0), 16, 18.0, 400, 0.05, 5.0),
                                         ((40, 20, 21), 0.5, (0.0, 0.0, 0.0), 8, 22.0, 260, 0.1, -1.0),
                                         ((1, 1, 1), 0.5, (0.0, 0.0, 0.0), 3, 5.0, 3, 0.2, 3.0)]:
        g.append(synth.Geometry(n[0], n[1], n[2], dx, synth.centred_origin(n[0], dx) + off[0],
                                synth.centred_origin(n[1], dx) + off[1],
                                synth.centred_origin(n[2], dx) + off[2],
                                synth.fibonacci_sphere(Q, Rs), K, dt, t0, 1.5, 1.0))
    return g


def test_host_fbp_window_bounds(tmp_path):
    """FBP reads samples floor(kt) and floor(kt) + 1 from a per-(tile,
    transducer) window of staged samples; the window must hold them for
    every voxel, tile and transducer of every workload (the kernel only
    clamps the index to stay inside its row)."""
    exe = tmp_path / "fbp_window_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_1304_2017_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "fbp_window_check.cpp"), "-o", str(exe)],
                   check=True)
    for geom in _fbp_window_workloads():
        lines = [" ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in
                          (geom.nx, geom.ny, geom.nz, float(geom.dx), float(geom.x0),
                           float(geom.y0), float(geom.z0), float(geom.c0), float(geom.dt),
                           float(geom.t0), geom.n_t, geom.n_det))]
        lines += [" ".join(repr(float(c)) for c in r) for r in geom.det_xyz]
        r = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True,
                           text=True, timeout=300)
        assert r.returncode == 0, (geom.name, r.stdout + r.stderr)
        assert r.stdout.startswith("OK"), (geom.name, r.stdout)
        pairs, lo_m, hi_m = map(int, r.stdout.split()[1:4])
        print(f"{geom.name or geom.shape}: {pairs} tile-transducer pairs, margins {lo_m} / {hi_m}")
        assert pairs > 0 and lo_m >= 0 and hi_m >= 0


def _fit_small_rot():
    import importlib.util
    path = os.path.join(ROOT, "paper_1304_2017_amd", "csrc", "fit_small_rot.py")
    spec = importlib.util.spec_from_file_location("fit_small_rot", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_small_rot_coefficients_match_their_fit():
    """The ring-point rotation's sin d and cos d - 1 polynomials (|d| <= pi/8)
    carry the coefficients that fit_small_rot.py derives (to 1 FP32 ulp), and
    their relative errors bound the position error: a point at ring radius r
    moves by r |d| err, at most 16 err cells for rings of 256 points or more
    (|d| <= 16 2 pi / N_j, r = N_j / 2 pi) and 40 (pi/8) err below that."""
    fit = _fit_small_rot()
    want = np.array(fit.coefficients(), dtype=np.float32)
    text = open(os.path.join(ROOT, "paper_1304_2017_amd", "csrc", "oat_geom.hpp")).read()
    body = text[text.index("OAT_HD void small_rot"):]
    body = body[:body.index("}")]
    lits = [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    # order in the source: a2, a1, 1.0, b2, b1, -0.5
    assert len(lits) == 6 and lits[2] == 1.0 and lits[5] == -0.5, lits
    got = np.array([lits[1], lits[0], lits[4], lits[3]], dtype=np.float32)
    ulp = np.spacing(np.abs(want))
    assert np.all(np.abs(got - want) <= ulp), (got, want)
    es, ec = fit.max_relative_errors(tuple(float(x) for x in got))
    assert es < 3e-8 and ec < 1e-8, (es, ec)
    assert 16 * es < 5e-7 and 40 * (np.pi / 8) * es < 5e-7
    # FP32 evaluation as the kernel does it (fmaf emulated in FP64, rounded)
    d = np.linspace(-np.pi / 8, np.pi / 8, 20001).astype(np.float32)
    f32 = np.float32

    def fma(a, b, c):
        return f32(np.float64(a) * np.float64(b) + np.float64(c))
    d2 = (d * d).astype(np.float32)
    sn = fma(d2, fma(d2, got[1], got[0]), f32(1.0)) * d
    cm1 = fma(d2, fma(d2, got[3], got[2]), f32(-0.5)) * d2
    dd = d.astype(np.float64)
    assert np.max(np.abs(sn - np.sin(dd))) < 1.5e-7 * np.pi / 8
    assert np.max(np.abs(cm1 + 2 * np.sin(dd / 2) ** 2)) < 2e-8
