"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances, each gated both as a relative L2 over the whole output and
element by element (max |error| / max |reference|, see checks.py): FP32
storage 1e-5 for H, H^T and FBP; G alone 5e-7 (D amplifies G's error about
12x at the 256^3 workload); BF16 output storage 2e-3 in L2 and half a BF16
ulp element-wise, with the oracle fed the same BF16-rounded inputs.
"""
import math
import sys

import numpy as np
import pytest

from checks import BF16_ELEM, check
from paper_1304_2017_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from oracle import ref  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev():
    return torch.device("cuda", 0)


def _t(x, dtype=torch.float32):
    return torch.tensor(np.asarray(x), dtype=torch.float64).to(dtype).to(_dev())


def _np(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _bf16_round(x):
    return torch.tensor(np.asarray(x)).to(torch.bfloat16).double().numpy()


@pytest.fixture(scope="module")
def Plan():
    from paper_1304_2017_amd.oat import Plan as P
    return P


def _small_case(seed, Plan):
    geom, balls, img = synth.config_small(seed)
    return geom, balls, img, Plan(geom, 0), seed


@pytest.fixture(scope="module", params=[0, 1, 2, 3, 4])
def small(request, Plan):
    return _small_case(request.param, Plan)


@pytest.fixture(scope="module", params=[0, 1])
def small_bf16(request, Plan):
    """Two seeds suffice for the BF16 storage checks."""
    return _small_case(request.param, Plan)


def test_bf16_image_box_gives_the_fp32_result(small_bf16):
    """G with a BF16 image keeps BF16 node pairs in its LDS box; the values
    are the image's own, so G equals G of the same values stored in FP32,
    bit for bit (both with the segment table, ragged bricks included)."""
    geom, _, img, plan, seed = small_bf16
    _say(f"[gpu] G bf16 pair box 32^3 seed {seed}")
    xb = _t(img, torch.bfloat16)
    gb = plan.project(xb, srt_only=True, out_dtype=torch.float32)
    gf = plan.project(xb.float().contiguous(), srt_only=True, out_dtype=torch.float32)
    assert torch.equal(gb, gf)


def test_srt_only_matches_oracle(small):
    geom, _, img, plan, seed = small
    _say(f"[gpu] G 32^3 seed {seed}")
    g = _np(plan.project(_t(img), srt_only=True))
    check("G", g, ref.srt(geom.as_dict(), img), 5e-7)


def test_project_matches_oracle(small):
    geom, _, img, plan, seed = small
    _say(f"[gpu] H 32^3 seed {seed}")
    p = _np(plan.project(_t(img)))
    check("H", p, ref.project(geom.as_dict(), img), 1e-5)


def test_backproject_matches_oracle(small):
    geom, _, _, plan, seed = small
    _say(f"[gpu] H^T 32^3 seed {seed}")
    rng = np.random.default_rng(100 + seed)
    y = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32).astype(np.float64)
    a = _np(plan.backproject(_t(y)))
    check("H^T", a, ref.backproject(geom.as_dict(), y), 1e-5)
    b = _np(plan.backproject(_t(y), srt_only=True))
    check("G^T", b, ref.srt_adj(geom.as_dict(), y), 1e-5)


def test_fbp_matches_oracle(small):
    geom, balls, img, plan, seed = small
    _say(f"[gpu] FBP 32^3 seed {seed}")
    p = synth.nwave_balls(geom, balls).astype(np.float32).astype(np.float64)
    f = _np(plan.fbp(_t(p)))
    check("FBP", f, ref.fbp(geom.as_dict(), p), 1e-5)


def test_fbp_floor_at_exact_sample_times(Plan):
    """Nodes whose FP64 sample position kt is an exact integer (c0 dt = 1/8
    mm, transducers on the axes 20 mm from a node-centred grid): the FP32 kt
    lands within its error bound of the integer and the FP64 floor decides.
    A wrong decision moves a term by half a sample difference, far above the
    element-wise bound used here."""
    n, dx = 33, 0.5
    o = synth.centred_origin(n, dx)
    det = np.array([[0, 0, 20.0], [0, 0, -20.0], [20.0, 0, 0], [-20.0, 0, 0],
                    [0, 20.0, 0], [0, -20.0, 0]])
    geom = synth.Geometry(n, n, n, dx, o, o, o, det, 300, 0.125, 0.0, 1.0, 1.0,
                          np.full(6, 4.0 * np.pi * 400.0 / 6))
    gd = geom.as_dict()
    x, y, z = geom.node_coords()
    kt = np.zeros((6,) + geom.shape)
    for q in range(6):
        d = np.sqrt((x - det[q, 0]) ** 2 + (y - det[q, 1]) ** 2 + (z - det[q, 2]) ** 2)
        kt[q] = (d / 1.0 - 0.0) / 0.125
    exact = int(np.count_nonzero(kt == np.floor(kt)))
    _say(f"[gpu] FBP at exact sample times: {exact} node-transducer pairs with integer kt")
    assert exact > 1000
    plan = Plan(geom, 0)
    rng = np.random.default_rng(11)
    pr = rng.normal(size=(6, 300)).astype(np.float32).astype(np.float64)
    f = _np(plan.fbp(_t(pr)))
    fr = ref.fbp(gd, pr)
    err = float(np.max(np.abs(f - fr)))
    _say(f"  max abs error {err:.3e} of max |f| {np.max(np.abs(fr)):.3e}")
    assert err <= 1e-5 * float(np.max(np.abs(fr)))


def test_adjoint_identity_on_gpu(small):
    geom, _, _, plan, seed = small
    _say(f"[gpu] adjoint 32^3 seed {seed}")
    rng = np.random.default_rng(200 + seed)
    x = _t(rng.normal(size=geom.shape))
    y = _t(rng.normal(size=(geom.n_det, geom.n_t)))
    Hx = plan.project(x)
    HTy = plan.backproject(y)
    torch.cuda.synchronize()
    lhs = float(torch.dot(Hx.double().ravel(), y.double().ravel()))
    rhs = float(torch.dot(x.double().ravel(), HTy.double().ravel()))
    scale = float(Hx.double().norm() * y.double().norm())
    _say(f"  |<Hx,y>-<x,H^T y>| / (|Hx||y|) = {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_bf16_storage(small_bf16):
    geom, balls, img, plan, seed = small_bf16
    _say(f"[gpu] BF16 32^3 seed {seed}")
    gd = geom.as_dict()
    img_b = _bf16_round(img)
    p = _np(plan.project(_t(img, torch.bfloat16), out_dtype=torch.bfloat16))
    check("H bf16", p, ref.project(gd, img_b), 2e-3, BF16_ELEM)
    rng = np.random.default_rng(300 + seed)
    y_b = _bf16_round(rng.normal(size=(geom.n_det, geom.n_t)))
    a = _np(plan.backproject(_t(y_b, torch.bfloat16), out_dtype=torch.bfloat16))
    check("H^T bf16", a, ref.backproject(gd, y_b), 2e-3, BF16_ELEM)
    pn = _bf16_round(synth.nwave_balls(geom, balls))
    f = _np(plan.fbp(_t(pn, torch.bfloat16), out_dtype=torch.bfloat16))
    check("FBP bf16", f, ref.fbp(gd, pn), 2e-3, BF16_ELEM)
    # mixed: BF16 image in, FP32 data out
    p2 = _np(plan.project(_t(img, torch.bfloat16), out_dtype=torch.float32))
    check("H bf16 in, f32 out", p2, ref.project(gd, img_b), 1e-5)


# ---------------------------------------------------------------------------
# Ragged grids, off-centre origins, t0 > 0, grids smaller than one brick, a
# single node with the fewest samples allowed (3), whole bricks plus one
# slice with samples at negative times (s = 0 there).
# ---------------------------------------------------------------------------
RAGGED = [
    dict(n=(37, 29, 23), dx=0.45, off=(0.3, -0.7, 0.2), Q=24, Rs=21.0, K=300, dt=0.08, t0=0.0),
    dict(n=(7, 5, 9), dx=0.8, off=(0.0, 0.0, 0.0), Q=10, Rs=15.0, K=200, dt=0.1, t0=2.0),
    dict(n=(41, 22, 3), dx=0.3, off=(-1.0, 0.5, 0.0), Q=16, Rs=18.0, K=400, dt=0.05, t0=5.0),
    dict(n=(1, 1, 1), dx=0.5, off=(0.0, 0.0, 0.0), Q=3, Rs=5.0, K=3, dt=0.2, t0=3.0),
    dict(n=(40, 20, 21), dx=0.5, off=(0.0, 0.0, 0.0), Q=8, Rs=22.0, K=260, dt=0.1, t0=-1.0),
]


TABLES = {"segments": dict(arc_table="auto", segment_table="auto"),
          "arcs": dict(arc_table="auto", segment_table=False),
          "bounds": dict(arc_table=False, segment_table=False)}


def _check_tables(st, table):
    """The plan holds exactly the table of its path (the segment table is
    built from the bounds walk, so a plan that has it builds no arc table)."""
    assert (st["segment_table_bytes"] > 0) == (table == "segments")
    assert (st["arc_table_bytes"] > 0) == (table == "arcs")


@pytest.mark.parametrize("table", list(TABLES))
@pytest.mark.parametrize("case", range(len(RAGGED)))
def test_ragged_grids(case, table, Plan):
    c = RAGGED[case]
    nx, ny, nz = c["n"]
    det = synth.fibonacci_sphere(c["Q"], c["Rs"])
    geom = synth.Geometry(nx, ny, nz, c["dx"], synth.centred_origin(nx, c["dx"]) + c["off"][0],
                          synth.centred_origin(ny, c["dx"]) + c["off"][1],
                          synth.centred_origin(nz, c["dx"]) + c["off"][2], det, c["K"], c["dt"],
                          c["t0"], 1.5, 1.3)
    _say(f"[gpu] ragged case {case} tables {table} {c}")
    gd = geom.as_dict()
    rng = np.random.default_rng(case)
    img = rng.uniform(0, 1, size=geom.shape)
    img = img.astype(np.float32).astype(np.float64)
    plan = Plan(geom, 0, **TABLES[table])
    _check_tables(plan.stats(), table)
    g = _np(plan.project(_t(img), srt_only=True))
    check("G", g, ref.srt(gd, img), 5e-7)
    p = _np(plan.project(_t(img)))
    check("H", p, ref.project(gd, img), 1e-5)
    y = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32).astype(np.float64)
    a = _np(plan.backproject(_t(y)))
    check("H^T", a, ref.backproject(gd, y), 1e-5)
    f = _np(plan.fbp(_t(y)))
    check("FBP", f, ref.fbp(gd, y), 1e-5)


def test_zero_inputs_and_overwrite(Plan):
    geom = synth.config_small(0)[0]
    plan = Plan(geom, 0)
    _say("[gpu] zero inputs")
    z_img = torch.zeros(geom.shape, device=_dev())
    z_dat = torch.zeros((geom.n_det, geom.n_t), device=_dev())
    out_d = torch.full((geom.n_det, geom.n_t), 7.0, device=_dev())
    out_i = torch.full(geom.shape, 7.0, device=_dev())
    plan.project(z_img, out=out_d)
    plan.backproject(z_dat, out=out_i)
    torch.cuda.synchronize()
    assert float(out_d.abs().max()) == 0.0
    assert float(out_i.abs().max()) == 0.0
    plan.fbp(z_dat, out=out_i)
    torch.cuda.synchronize()
    assert float(out_i.abs().max()) == 0.0


def test_repeat_runs(Plan):
    """H sums its brick partials in a fixed order and H^T accumulates exact
    fixed-point integers (order-independent), so both are bit-stable."""
    geom, _, img, plan, seed = _small_case(0, Plan)
    _say("[gpu] repeat runs")
    x = _t(img)
    a = plan.project(x).clone()
    b = plan.project(x).clone()
    y = torch.randn((geom.n_det, geom.n_t), device=_dev())
    c = plan.backproject(y).clone()
    d = plan.backproject(y).clone()
    f1 = plan.fbp(y).clone()
    f2 = plan.fbp(y).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(c, d)
    assert torch.equal(f1, f2)
    # OAT_FLAG_DETERMINISTIC is accepted and changes nothing
    from paper_1304_2017_amd import oat
    L, h, s0 = oat.lib(), plan._h, oat.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out_d = torch.empty_like(a)
    out_i = torch.empty_like(c)
    out_f = torch.empty_like(f1)
    P = lambda t: oat.ctypes.c_void_p(t.data_ptr())
    assert L.oat_project(h, P(x), oat.OAT_F32, P(out_d), oat.OAT_F32,
                         oat.OAT_FLAG_DETERMINISTIC, s0) == oat.OAT_OK
    assert L.oat_backproject(h, P(y), oat.OAT_F32, P(out_i), oat.OAT_F32,
                             oat.OAT_FLAG_DETERMINISTIC, s0) == oat.OAT_OK
    assert L.oat_fbp(h, P(y), oat.OAT_F32, P(out_f), oat.OAT_F32,
                     oat.OAT_FLAG_DETERMINISTIC, s0) == oat.OAT_OK
    assert L.oat_fbp(h, P(y), oat.OAT_F32, P(out_f), oat.OAT_F32, 4, s0) == oat.OAT_ERR_ARG
    torch.cuda.synchronize()
    assert torch.equal(out_d, a) and torch.equal(out_i, c) and torch.equal(out_f, f1)


@pytest.mark.parametrize("seed", [0, 3])
def test_table_paths_agree(seed, Plan):
    """The plan's segment table, its arc table (tight arcs of the owned
    points) and the kernels' own arc bounds enumerate the same points: G
    agrees to FP32 summation order, G^T bit for bit (the same integer terms
    and the same calibrated scales), and all match the oracle."""
    geom, _, img = synth.config_small(seed)
    _say(f"[gpu] segment table vs arc table vs arc bounds seed {seed}")
    ps = Plan(geom, 0, **TABLES["segments"])
    pt = Plan(geom, 0, **TABLES["arcs"])
    pn = Plan(geom, 0, **TABLES["bounds"])
    ss, st, sn = ps.stats(), pt.stats(), pn.stats()
    _check_tables(ss, "segments")
    _check_tables(st, "arcs")
    _check_tables(sn, "bounds")
    assert ss["segment_table_entries"] > 0 and st["arc_table_entries"] > 0
    # budgets too small for the table: the next path
    assert Plan(geom, 0, arc_table=1, segment_table=False).stats()["arc_table_bytes"] == 0
    s1 = Plan(geom, 0, segment_table=1).stats()
    assert s1["segment_table_bytes"] == 0 and s1["arc_table_bytes"] > 0
    # the segment table needs no arc table
    s2 = Plan(geom, 0, arc_table=False).stats()
    assert s2["segment_table_bytes"] > 0 and s2["arc_table_bytes"] == 0
    x = _t(img)
    gs, gt, gn = (_np(p.project(x, srt_only=True)) for p in (ps, pt, pn))
    e1, e2 = rel(gs, gn), rel(gt, gn)
    _say(f"  G segments vs bounds rel {e1:.3e}, arcs vs bounds rel {e2:.3e}")
    assert e1 < 5e-7 and e2 < 5e-7
    check("G bounds path", gn, ref.srt(geom.as_dict(), img), 5e-7)
    rng = np.random.default_rng(400 + seed)
    y = _t(rng.normal(size=(geom.n_det, geom.n_t)))
    a_s, a_t, a_n = (_np(p.backproject(y, srt_only=True)) for p in (ps, pt, pn))
    _say(f"  G^T segments vs bounds rel {rel(a_s, a_n):.3e}, arcs vs bounds rel {rel(a_t, a_n):.3e}")
    assert np.array_equal(a_s, a_n) and np.array_equal(a_t, a_n)


def test_backproject_with_wide_dynamic_range(Plan):
    """The fixed-point scale of G^T follows the largest |D^T y|: one
    transducer 1e4 times louder than the others, and data of magnitude 1e-30,
    still match the oracle."""
    geom = synth.config_small(0)[0]
    plan = Plan(geom, 0)
    gd = geom.as_dict()
    rng = np.random.default_rng(31)
    y = rng.normal(size=(geom.n_det, geom.n_t))
    y[5] *= 1e4
    y = y.astype(np.float32).astype(np.float64)
    _say("[gpu] H^T with one loud transducer, and with 1e-30 data")
    check("H^T loud", _np(plan.backproject(_t(y))), ref.backproject(gd, y), 1e-5)
    tiny = (rng.normal(size=(geom.n_det, geom.n_t)) * 1e-30).astype(np.float32).astype(np.float64)
    check("H^T 1e-30", _np(plan.backproject(_t(tiny))), ref.backproject(gd, tiny), 1e-5)


def test_project_with_wide_dynamic_range(Plan):
    """G's shell sums are 64-bit fixed point with a power-of-two scale from
    each brick's largest |node|: images of magnitude 1e-30 and 1e30 still
    match the oracle, and a NaN node turns sums into NaN rather than into
    finite values."""
    geom, _, img = synth.config_small(2)
    plan = Plan(geom, 0)
    gd = geom.as_dict()
    for s in (1e-30, 1e30):
        x = (img * s).astype(np.float32).astype(np.float64)
        _say(f"[gpu] G with the image times {s:g}")
        check(f"G x{s:g}", _np(plan.project(_t(x), srt_only=True)), ref.srt(gd, x), 5e-7)
    x = img.astype(np.float32).copy()
    x[geom.nz // 2, geom.ny // 2, geom.nx // 2] = np.nan
    _say("[gpu] G with one NaN node")
    g = _np(plan.project(_t(x), srt_only=True))
    assert np.isnan(g).any()


@pytest.fixture(scope="module")
def small1_plan(Plan):
    """config_small's grid with 300 transducers: three windows of 128."""
    g = synth.config_small(1)[0]
    geom = synth.Geometry(g.nx, g.ny, g.nz, g.dx, g.x0, g.y0, g.z0,
                          synth.fibonacci_sphere(300, 25.0), g.n_t, g.dt, g.t0, g.c0, g.gamma)
    return geom, Plan(geom, 0)


@pytest.mark.parametrize("q", [0, 15, 16, 127, 128, 255, 256, 299])
def test_backproject_single_transducer(q, small1_plan):
    """Data on one transducer only, at every position class of G^T's
    transducer windows of 128 (first transducer, the ends of the first 16
    that the waves take, last of a window, first of the next, the partial
    last window): each window's scale must see that transducer's data."""
    geom, plan = small1_plan
    rng = np.random.default_rng(100 + q)
    y = np.zeros((geom.n_det, geom.n_t))
    y[q] = rng.normal(size=geom.n_t).astype(np.float32)
    _say(f"[gpu] H^T data on transducer {q}")
    check("H^T", _np(plan.backproject(_t(y))),
          ref.backproject(geom.as_dict(), y[q:q + 1], rows=np.array([q], dtype=np.int32)), 1e-5)


def _brick_slices(nbricks, items, min_items):
    """The library's slice count for a brick's work (G: transducers, G^T:
    windows of 128 transducers), restated to check that a case uses slices."""
    best, best_eff = 1, 0.0
    for sl in range(1, 5):
        if sl > 1 and items // sl < min_items:
            break
        g = nbricks * sl
        eff = g / (((g + 255) // 256) * 256)
        if eff > best_eff + 0.005:
            best, best_eff = sl, eff
    per = (items + best - 1) // best
    return (items + per - 1) // per


def _fill_slices(nbricks, items, min_items, max_slices, rnd):
    """The library's slice count for G on the segment table (rounds of 512)
    and for G^T (rounds of 256), restated: the best-filling count of up to
    max_slices, a larger count winning ties within 0.5%."""
    best, best_eff = 1, 0.0
    for c in range(1, max_slices + 1):
        if c > 1 and items // c < min_items:
            break
        per = (items + c - 1) // c
        n = (items + per - 1) // per
        g = nbricks * n
        eff = g / (((g + rnd - 1) // rnd) * rnd)
        if eff >= best_eff - 0.005:
            best, best_eff = n, max(eff, best_eff)
    return best


@pytest.mark.parametrize("table", list(TABLES))
def test_transducer_slices(table, Plan):
    """8 bricks and 768 transducers: G takes each brick's transducers in 8
    workgroups on the segment table and 4 on the other paths, and G^T its 6
    windows (of 128) in 3, each with its own FP64 brick sums added in slice
    order.  Parity with the oracle, and G^T bit-identical across the table
    paths."""
    geom0 = synth.config_small(1)[0]
    det = synth.fibonacci_sphere(768, 25.0)
    geom = synth.Geometry(geom0.nx, geom0.ny, geom0.nz, geom0.dx, geom0.x0, geom0.y0, geom0.z0,
                          det, geom0.n_t, geom0.dt, geom0.t0, geom0.c0, 1.0)
    assert _fill_slices(8, 768, 64, 8, 512) == 8 and _brick_slices(8, 768, 64) == 4
    assert _fill_slices(8, 768 // 128, 2, 8, 256) == 3
    _say(f"[gpu] transducer slices, tables {table}")
    gd = geom.as_dict()
    rng = np.random.default_rng(21)
    img = rng.uniform(0, 1, size=geom.shape).astype(np.float32).astype(np.float64)
    y = rng.normal(size=(geom.n_det, geom.n_t)).astype(np.float32).astype(np.float64)
    plan = Plan(geom, 0, **TABLES[table])
    g = _np(plan.project(_t(img), srt_only=True))
    check("G", g, ref.srt(gd, img), 5e-7)
    a = _np(plan.backproject(_t(y), srt_only=True))
    check("G^T", a, ref.srt_adj(gd, y), 1e-5)
    lhs = float(np.dot(g.ravel(), y.ravel()))
    rhs = float(np.dot(img.ravel(), a.ravel()))
    scale = float(np.linalg.norm(g) * np.linalg.norm(y))
    _say(f"  adjoint (/ norms) {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= 1e-6 * scale
    if table == "segments":
        a_b = _np(Plan(geom, 0, **TABLES["bounds"]).backproject(_t(y), srt_only=True))
        assert np.array_equal(a, a_b)
