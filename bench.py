"""Benchmark of the hot path on one MI355X.

One step = H (project), H^T (backproject) and FBP once each on the
256^3 / 2048-transducer / 1024-sample workload (0.1 mm voxels, 40 seeded
ellipsoids, Fibonacci hemisphere of radius 40 mm, 20 MHz, FP32 storage).
Each operator performs N*Q voxel-view updates.  The headline value is the
H/H^T rate, 2*N*Q / (t_H + t_HT) from the operators' own HIP-event times over
the timed steps; FBP is timed in the same steps and reported under "ops".

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X FP32 vector peak, 157.3 TFLOP/s (256 CUs at 2.4 GHz), with an FMA
# counted as one lane-op: 7.86e13 lane-ops/s.  (A CU issues more than one
# wave64 VALU instruction per cycle: the FBP kernel measures 1.24.)
VALU_PEAK = 157.3e12 / 2
HBM_PEAK = 8.0e12   # bytes/s
BF16_PEAK = 2.5e15  # dense BF16 matrix-core FLOP/s
# Algorithmic FP32 VALU operations of one quadrature point of G or G^T
# (position 6 FMA, cos/sin of the azimuth 2 transcendental = 8 issue slots,
# floor 3, fraction 3, cell address 3, trilinear 7 lerps = 14, weighted add 2).
OPS_PER_POINT = 39
# Algorithmic VALU operations of one FBP voxel-view update (difference 3,
# squared norm 3, rsqrt 4, distance/kt 2, floor 2, two coefficients 4,
# two-term sum 2, weighted add 1).
OPS_PER_FBP_UPDATE = 21


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256cube.txt")


# Sources of the kernels the default line measures (G, G^T, FBP, D, D^T, the
# brick-sum gather and the plan's tables), with the headers they include.
SRT_SOURCES = ("oat_srt.hip", "oat_aux.hip", "oat_plan.cpp", "oat_internal.hpp", "oat_geom.hpp",
               "oat_dtype.hpp", "oat_fbp_window.hpp", "oat_fbp_floor.hpp")


def kernel_sources_sha256():
    """Hash of the HIP/C++ sources of the measured kernels (SRT_SOURCES and
    include/oat.h): a counter summary taken with other sources no longer
    describes them."""
    import hashlib
    d = os.path.join(ROOT, "paper_1304_2017_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(SRT_SOURCES):
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(ROOT, "include", "oat.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a device copy of known size),
    or None when the summary is missing or the kernel sources have changed
    since the counters were taken."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    fields = {}
    for ln in lines:
        t = ln.split()
        if len(t) >= 2 and not ln.startswith("#"):
            fields.setdefault(t[0], []).append(t[1:])
    if fields.get("sources", [[None]])[0][0] != kernel_sources_sha256():
        return None
    for t in fields.get("kernel", []):
        if t[0] == kernel:
            kv = dict(zip(t[1::2], t[2::2]))
            return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


def quad_points(geom):
    """Quadrature points that one G or G^T pass evaluates: every cell of the
    footprint [-1, n-1]^3 is crossed by dx/(c0 dt) points per transducer
    (shell spacing c0 dt, point spacing dx on each shell)."""
    cells = (geom.nx + 1) * (geom.ny + 1) * (geom.nz + 1)
    return cells * geom.n_det * geom.dx / (geom.c0 * geom.dt)


def cpu_baseline(geom, img, p_np):
    """Time the FP64 oracle on a bounded sample of the same workload and
    scale to voxel-view updates per second of H and H^T (the headline
    metric), as the paper extrapolated its CPU times from a subset of
    transducers.  H and H^T run on every 64th transducer (32 rows): each
    oracle call has a fixed cost (H^T allocates, clears and sums one FP64
    image per thread), which a sample of 32 rows keeps small against the
    rows' own work instead of multiplying it by Q.  FBP is timed on 200000
    voxels and reported beside it."""
    from oracle import ref
    gd = geom.as_dict()
    N, Q = geom.n_vox, geom.n_det
    rows = np.arange(0, Q, 64, dtype=np.int32)           # 32 transducers
    t = time.perf_counter()
    ref.project(gd, img, rows=rows)
    t_h = (time.perf_counter() - t) * Q / rows.size
    t = time.perf_counter()
    ref.backproject(gd, p_np[rows], rows=rows)
    t_ht = (time.perf_counter() - t) * Q / rows.size
    rng = np.random.default_rng(0)
    vox = rng.choice(N, 200000, replace=False)
    t = time.perf_counter()
    ref.fbp(gd, p_np, voxels=vox)
    t_f = (time.perf_counter() - t) * N / vox.size
    cores = ref.max_threads()
    # The same on one thread, on a smaller sample (the paper's CPU code was sequential).
    ref.set_threads(1)
    try:
        r1 = rows[:1]
        t = time.perf_counter()
        ref.project(gd, img, rows=r1)
        t1_h = (time.perf_counter() - t) * Q
        t = time.perf_counter()
        ref.backproject(gd, p_np[r1], rows=r1)
        t1_ht = (time.perf_counter() - t) * Q
        v1 = vox[:2000]
        t = time.perf_counter()
        ref.fbp(gd, p_np, voxels=v1)
        t1_f = (time.perf_counter() - t) * N / v1.size
    finally:
        ref.set_threads(cores)
    return dict(value=2.0 * N * Q / (t_h + t_ht), unit="voxel-view updates/s",
                cores=cores, kind="oracle",
                sample=(f"H and H^T on every 64th of {Q} transducers ({rows.size} rows), "
                        f"FBP on {vox.size} of {N} voxels; times scaled linearly to the "
                        f"full operators (extrapolated s: H {t_h:.0f}, H^T {t_ht:.0f}, "
                        f"FBP {t_f:.0f}); one thread: H and H^T on 1 transducer, FBP on "
                        f"2000 voxels (extrapolated s: H {t1_h:.0f}, H^T {t1_ht:.0f}, "
                        f"FBP {t1_f:.0f})"),
                extrapolated_s=dict(H=t_h, HT=t_ht, FBP=t_f),
                FBP_updates_per_s=N * Q / t_f,
                value_1thread=2.0 * N * Q / (t1_h + t1_ht),
                extrapolated_1thread_s=dict(H=t1_h, HT=t1_ht, FBP=t1_f))


def time_op(fn, reps, warm=1):
    """Median wall time (s) of fn over reps runs after warm runs, each
    bracketed by HIP events on the current stream."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    return float(np.median(ts))


def pls_run(cfg, iters):
    """PLS-TV (smoothed isotropic TV, nonlinear CG) from a = 0 on the 192^3 /
    4096-transducer N-wave data (cfg "c") or on H a_true + 1% noise at the
    256^3 / 8192-transducer workload (cfg "e"), with FP32 and BF16 operator
    storage.  Prints one JSON line per storage type."""
    import torch
    from paper_1304_2017_amd import recon, synth
    from paper_1304_2017_amd.oat import Plan
    if cfg == "c":
        geom, balls, u_np = synth.config_c(0)
        plan = Plan(geom, 0)
        u = torch.from_numpy(u_np.astype(np.float32)).cuda()
        phantom = torch.from_numpy(synth.voxelise_balls(geom, balls).astype(np.float32)).cuda()
    else:
        geom, _, img = synth.config_e(0)
        plan = Plan(geom, 0)
        phantom = torch.from_numpy(img).cuda()
        clean = plan.project(phantom)
        torch.cuda.synchronize()
        gen = torch.Generator(device="cuda").manual_seed(0)
        u = clean + 0.01 * float(clean.abs().max()) * torch.randn(clean.shape, device="cuda",
                                                                   generator=gen)
    # eps: 1e-3 of the largest image value one expects (amplitudes <= 1);
    # mu: the penalty of the zero image is 0.1% of ||u||^2.
    eps = 1e-3
    mu = 1e-3 * float(u.double().pow(2).sum()) / (geom.n_vox * eps)
    for dt in (torch.float32, torch.bfloat16):
        recon.pls_tv(plan, u, mu=mu, eps=eps, iters=1, storage=dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = recon.pls_tv(plan, u, mu=mu, eps=eps, iters=iters, storage=dt, track=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        f = plan.fbp(u.to(dt), out_dtype=dt)
        print(json.dumps(dict(workload=geom.name, storage=str(dt).split(".")[-1], iters=iters,
                              mu=mu, eps=eps, seconds=el, s_per_iter=el / iters,
                              rmse=recon.rmse(res.image, phantom),
                              fbp_rmse=recon.rmse(f.float(), phantom),
                              phantom_rms=recon.rmse(torch.zeros_like(phantom), phantom),
                              residuals=[round(v, 6) for v in res.residuals],
                              objective=[float("%.8g" % v) for v in res.objective])), flush=True)
    plan.close()


def paper_run(iters):
    """The paper's simulation study at its shape (Sec. IV.A; Sec. V.B): the
    210 x 210 x 440 grid at 0.14 mm, 9 Gaussian-blurred spheres, the
    N-wave of the spheres blurred in time (FWHM 0.5 us) on 32x45, 64x45,
    64x90 and 128x90 ring views at 65 mm, 1022 samples at 20 MHz from
    17.5 us.  For each data set and for FP32 and BF16 operator storage: FBP
    and PLS-Int (linear CG, mu = 0 as in the simulation study, `iters`
    iterations from 0), their times and the RMSE of Sec. IV.A against the
    phantom.  Prints one JSON line per data set and storage."""
    import torch
    from paper_1304_2017_amd import recon, synth
    from paper_1304_2017_amd.oat import Plan
    t0 = time.perf_counter()
    _, balls, phantom = synth.config_p(0)
    ph = torch.from_numpy(phantom).cuda()
    log(f"[paper] phantom in {time.perf_counter() - t0:.1f} s")
    for nr, nv in ((32, 45), (64, 45), (64, 90), (128, 90)):
        geom = synth.config_p_rings(nr, nv)
        u = torch.from_numpy(synth.config_p_data(geom, balls).astype(np.float32)).cuda()
        t0 = time.perf_counter()
        # the 128x90 table (~180 GB) needs more than the default 40% of the
        # free memory: this run dedicates the device to the reconstruction
        free, _ = torch.cuda.mem_get_info()
        plan = Plan(geom, 0, segment_table=int(0.75 * free)) if nr * nv > 5760 else Plan(geom, 0)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        st = plan.stats()
        for dt in (torch.float32, torch.bfloat16):
            ud = u.to(dt)
            f = plan.fbp(ud, out_dtype=dt)
            t_fbp = time_op(lambda: plan.fbp(ud, out_dtype=dt), 3)
            res = recon.pls_cg(plan, u, mu=0.0, iters=iters, storage=dt)
            torch.cuda.synchronize()
            per_it = (res.times[-1] - res.times[0]) / max(len(res.times) - 1, 1)
            fresh = float((u - plan.project(res.image)).double().norm() / u.double().norm())
            print(json.dumps(dict(
                workload=geom.name, views=f"{nr}x{nv}", transducers=geom.n_det,
                storage="f32" if dt == torch.float32 else "bf16",
                fbp_ms=t_fbp * 1e3, fbp_rmse=recon.rmse(f.float(), ph),
                pls_iterations=len(res.residuals) - 1, pls_s_per_iteration=per_it,
                pls_rmse=recon.rmse(res.image, ph), pls_residual=res.residuals[-1],
                pls_fresh_residual=fresh, phantom_rms=recon.rmse(torch.zeros_like(ph), ph),
                plan_s=plan_s, segment_table_bytes=st["segment_table_bytes"],
                arc_table_bytes=st["arc_table_bytes"])), flush=True)
            log(f"[paper] {nr}x{nv} {dt}: FBP {t_fbp * 1e3:.1f} ms, PLS-Int {per_it:.3f} s/it, "
                f"RMSE FBP {recon.rmse(f.float(), ph):.4f} PLS {recon.rmse(res.image, ph):.4f}")
            del f, res, ud
        plan.close()
        del plan, u
        torch.cuda.empty_cache()


def learned_run(n_phantoms, epochs, iters):
    """Time-to-residual of PLS-TV, plain vs learned preconditioner, at the
    256^3 / 8192-sphere workload (data H a_true + 1% noise).  The network is
    trained first (time reported separately) on (gradient, error) pairs from
    10 plain iterations per seeded 128^3 / 1024-transducer phantom.  r* is the
    plain residual after `iters` iterations; the learned run stops at r*.
    Prints one JSON line."""
    import torch
    from paper_1304_2017_amd import precond, recon, synth
    from paper_1304_2017_amd.oat import Plan
    t0 = time.perf_counter()
    gd, phantoms = synth.config_d_phantoms(n_phantoms, seed=1)
    t_phantoms = time.perf_counter() - t0
    log(f"[learned] {len(phantoms)} phantoms in {t_phantoms:.1f} s")
    plan_d = Plan(gd, 0)
    t0 = time.perf_counter()
    pairs = precond.training_pairs(plan_d, [torch.from_numpy(p) for p in phantoms], iters=10)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    plan_d.close()
    del phantoms
    log(f"[learned] {len(pairs)} pairs in {t_pairs:.1f} s")
    model = precond.Preconditioner(seed=0)
    t0 = time.perf_counter()
    tl = precond.train(model, pairs, epochs=epochs, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n = len(pairs)
    loss_first, loss_last = float(np.mean(tl.loss[:n])), float(np.mean(tl.loss[-n:]))
    log(f"[learned] trained {epochs} epochs in {t_train:.1f} s; loss {loss_first:.4f} -> {loss_last:.4f}")
    del pairs
    torch.cuda.empty_cache()

    geom, _, img = synth.config_e(0)
    plan = Plan(geom, 0)
    st = plan.stats()
    log(f"[learned] plan: segment table {st['segment_table_bytes'] / 1e9:.1f} GB, "
        f"arc table {st['arc_table_bytes'] / 1e9:.1f} GB")
    clean = plan.project(torch.from_numpy(img).cuda())
    torch.cuda.synchronize()
    gen = torch.Generator(device="cuda").manual_seed(0)
    u = clean + 0.01 * float(clean.abs().max()) * torch.randn(clean.shape, device="cuda", generator=gen)
    eps = 1e-3
    mu = 1e-3 * float(u.double().pow(2).sum()) / (geom.n_vox * eps)
    phantom = torch.from_numpy(img).cuda()
    recon.pls_tv(plan, u, mu=mu, eps=eps, iters=1)          # warm-up
    torch.cuda.synchronize()
    # image RMSE of every iterate, taken after its time is recorded
    rmse_plain, rmse_learned = [], []
    plain = recon.pls_tv(plan, u, mu=mu, eps=eps, iters=iters,
                         observe=lambda k, a: rmse_plain.append(recon.rmse(a, phantom)))
    torch.cuda.synchronize()
    # targets: the plain residual after 5, 10, 20 and `iters` iterations
    marks = sorted({k for k in (5, 10, 20, iters) if k <= iters})
    targets = {k: plain.residuals[k] for k in marks}
    r_star = targets[iters]
    log(f"[learned] plain {iters} iterations {plain.times[-1]:.1f} s, r* = {r_star:.5f}")
    # The learned iteration runs `iters` iterations too (no early stop): its
    # time to each target is the time of the first iterate below it, as if it
    # had stopped there, and the later iterates show where it goes on to.
    learned = precond.pls_tv_learned(plan, u, model, mu=mu, eps=eps, iters=iters,
                                     observe=lambda k, a: rmse_learned.append(recon.rmse(a, phantom)))
    torch.cuda.synchronize()

    def first(vals, times, r):
        k = next((i for i, v in enumerate(vals) if v <= r), None)
        return (k, times[k] if k is not None else None)

    def compare(vals_p, vals_l, key):
        out = []
        for k in marks:
            r = vals_p[k]
            kp, tp = first(vals_p, plain.times, r)
            kl, tl_ = first(vals_l, learned.times, r)
            out.append({"plain_iterations_for_target": k, "target": r, "plain_iterations": kp,
                        "plain_s": tp, "learned_iterations": kl, "learned_s": tl_,
                        "speedup": (tp / tl_) if (tp and tl_) else None,
                        "plain_rmse": rmse_plain[kp] if kp is not None else None,
                        "learned_rmse": rmse_learned[kl] if kl is not None else None,
                        "key": key})
        return out

    per_target = compare(plain.residuals, learned.residuals, "residual")
    log(f"[learned] r* reached by the learned iteration at iterate "
        f"{per_target[-1]['learned_iterations']} ({per_target[-1]['learned_s']} s)")
    # the same comparison on the PLS-TV objective ||u - H a||^2 + mu TV_eps(a)
    per_objective = compare(plain.objective, learned.objective, "objective")
    # the recursive residual checked by one fresh H on each final image
    unorm = float(u.double().norm())

    def fresh(a):
        return float((u - plan.project(a.float().contiguous())).double().norm()) / unorm

    f_fbp = plan.fbp(u)

    print(json.dumps(dict(
        workload=geom.name, data="H a_true + 1% noise, 60 seeded ellipsoids", mu=mu, eps=eps,
        plan=dict(segment_table_bytes=st["segment_table_bytes"],
                  arc_table_bytes=st["arc_table_bytes"]),
        r_star=r_star, targets=per_target, objective_targets=per_objective,
        rmse=dict(plain=recon.rmse(plain.image, phantom), learned=recon.rmse(learned.image, phantom),
                  fbp=recon.rmse(f_fbp, phantom),
                  phantom_rms=recon.rmse(torch.zeros_like(phantom), phantom)),
        plain=dict(iterations=len(plain.residuals) - 1, seconds=plain.times[-1],
                   fresh_residual=fresh(plain.image),
                   residuals=[round(v, 6) for v in plain.residuals],
                   objective=[float(v) for v in plain.objective],
                   rmse=[round(v, 6) for v in rmse_plain],
                   times=[round(v, 4) for v in plain.times]),
        learned=dict(iterations=len(learned.residuals) - 1, seconds=learned.times[-1],
                     directions=[(k, round(c, 4)) for k, c in learned.directions],
                     reached=min(learned.residuals) <= r_star,
                     seconds_to_r_star=per_target[-1]["learned_s"],
                     fresh_residual=fresh(learned.image),
                     residuals=[round(v, 6) for v in learned.residuals],
                     objective=[float(v) for v in learned.objective],
                     rmse=[round(v, 6) for v in rmse_learned],
                     times=[round(v, 4) for v in learned.times]),
        training=dict(workload=gd.name, phantoms=n_phantoms, pairs=n, epochs=epochs,
                      phantom_s=t_phantoms, pairs_s=t_pairs, train_s=t_train,
                      loss_first_epoch=loss_first, loss_last_epoch=loss_last))), flush=True)


def eir_run(reps):
    """H and H^T with a 64-tap EIR (Eq. (EIR)), and the Hann-window
    deconvolution (f_c = 5 MHz) followed by FBP, at the 256^3 / 2048 / 1024
    workload; one JSON line."""
    import torch
    from paper_1304_2017_amd import synth
    from paper_1304_2017_amd.oat import Plan
    geom, _, img = synth.config_large(0, dtype=np.float32)
    plan = Plan(geom, 0)
    x = torch.from_numpy(img).cuda()
    p = torch.empty(plan.data_shape, device="cuda")
    a = torch.empty(plan.image_shape, device="cuda")
    d = torch.empty(plan.data_shape, device="cuda")
    t_h0 = time_op(lambda: plan.project(x, out=p), reps)
    t_ht0 = time_op(lambda: plan.backproject(p, out=a), reps)
    h = synth.gamma_pulse(64, geom.dt, 0.1)
    plan.set_eir(h)
    t_h = time_op(lambda: plan.project(x, out=p), reps)
    t_ht = time_op(lambda: plan.backproject(p, out=a), reps)
    t_dec = time_op(lambda: plan.deconvolve(p, 5.0, out=d), reps)
    t_fbp = time_op(lambda: plan.fbp(d, out=a), reps)
    print(json.dumps(dict(
        workload="256^3 / 2048 transducers / 1024 samples, 64-tap gamma-pulse EIR (tau 0.1 us)",
        H_ms=t_h * 1e3, HT_ms=t_ht * 1e3, H_no_eir_ms=t_h0 * 1e3, HT_no_eir_ms=t_ht0 * 1e3,
        deconvolve_ms=t_dec * 1e3, fbp_ms=t_fbp * 1e3, fft_length=2 * 1024, f_cut_mhz=5.0,
        reps=reps)), flush=True)


def sph_run(reps):
    """The spherical-voxel model (25.6 mm field of view, 2048 hemisphere
    transducers, 256 frequencies in (0, 5] MHz) at 64^3 and 128^3, with
    point-like transducers and with 2 x 2 mm faces (4 x 4 Gauss-Legendre
    nodes, Sec. IV.B's transducer size): H_sph and H_sph^T times, terms per
    second (one term = one (voxel, frequency, face node) of one transducer)
    and the fraction of the VALU peak at 6 operations per term (a complex
    rotation and a weighted complex add).  One JSON line per case."""
    import torch
    from paper_1304_2017_amd import synth
    from paper_1304_2017_amd.oat import Plan
    n_f, df = 256, 5.0 / 256
    for n in (64, 128):
        geom, img = synth.config_sph(n=n)
        plan = Plan(geom, 0, arc_table=False, segment_table=False)
        x = torch.from_numpy(img).cuda()
        u = torch.empty((geom.n_det, n_f), device="cuda", dtype=torch.complex64)
        a = torch.empty(plan.image_shape, device="cuda")
        nnz = int(np.count_nonzero(img))
        for face in ((0.0, 0.0, 1), (2.0, 2.0, 4)):
            plan.set_aperture(*face)
            nodes = face[2] ** 2 if face[0] > 0 else 1
            t_f = time_op(lambda: plan.sph_project(x, n_f, df, df, out=u), reps)
            t_b = time_op(lambda: plan.sph_backproject(u, df, df, out=a), reps)
            terms_f = float(nnz) * geom.n_det * n_f * nodes
            terms_b = float(geom.n_vox) * geom.n_det * n_f * nodes
            print(json.dumps(dict(
                workload=f"{n}^3 ({25.6 / n:.2f} mm), 2048 hemisphere transducers, 256 frequencies "
                         "f_l = (l+1) * 5/256 MHz",
                faces="point-like" if nodes == 1 else f"{face[0]} x {face[1]} mm, {face[2]}x{face[2]} nodes",
                H_sph_ms=t_f * 1e3, H_sph_T_ms=t_b * 1e3, nonzero_voxels=nnz, voxels=geom.n_vox,
                H_sph_terms_per_s=terms_f / t_f, H_sph_T_terms_per_s=terms_b / t_b,
                H_sph_valu_frac=6 * terms_f / t_f / VALU_PEAK,
                H_sph_T_valu_frac=6 * terms_b / t_b / VALU_PEAK, reps=reps)), flush=True)
            log(f"[sph] {n}^3 faces {face}: H_sph {t_f * 1e3:.1f} ms, H_sph^T {t_b * 1e3:.1f} ms")
        plan.close()
        del plan, x, u, a
        torch.cuda.empty_cache()


def cnn_run(reps):
    """The learned preconditioner's BF16 16 -> 16 convolution on the matrix
    cores (forward, which also serves the data backward, and the weight
    gradient) at 128^3 and 256^3, against the 2.5 PFLOP/s dense BF16 peak,
    beside the FP32-activation VALU kernel and one whole network forward
    (1 -> 16 -> 16 -> 1 layers) in BF16.  Prints one JSON line."""
    import torch
    from paper_1304_2017_amd import precond
    out = []
    g = torch.Generator(device="cuda").manual_seed(0)
    model = precond.Preconditioner(seed=0)
    for n in (128, 256):
        x = torch.randn((16, n, n, n), device="cuda", generator=g).to(torch.bfloat16)
        dy = torch.randn((16, n, n, n), device="cuda", generator=g).to(torch.bfloat16)
        w = torch.randn((16, 16, 27), device="cuda", generator=g) * 0.1
        b = torch.zeros((16,), device="cuda")
        flop = 2.0 * n ** 3 * 16 * 16 * 27
        t_f = time_op(lambda: precond.conv3d(x, w, b, relu=True), reps)
        t_w = time_op(lambda: precond.conv3d_weight_grad(x, dy), reps)
        x32 = x.float()
        t_v = time_op(lambda: precond.conv3d(x32, w, b, relu=True), max(1, reps // 2))
        v = torch.randn((n, n, n), device="cuda", generator=g)
        t_m = time_op(lambda: model.forward(v), reps)
        # activation traffic of one bf16 16 -> 16 layer: 16 channels in, 16 out
        io_bytes = 2.0 * 2 * 16 * n ** 3
        out.append(dict(
            shape=f"{n}^3", flop_per_layer=flop,
            fwd_ms=t_f * 1e3, fwd_tflops=flop / t_f / 1e12, fwd_frac_bf16_peak=flop / t_f / BF16_PEAK,
            fwd_hbm_frac=io_bytes / t_f / HBM_PEAK,
            wgrad_ms=t_w * 1e3, wgrad_tflops=flop / t_w / 1e12,
            wgrad_frac_bf16_peak=flop / t_w / BF16_PEAK,
            fp32_valu_fwd_ms=t_v * 1e3, fp32_valu_tflops=flop / t_v / 1e12,
            network_forward_ms=t_m * 1e3))
        log(f"[cnn] {n}^3: fwd {t_f * 1e3:.3f} ms ({flop / t_f / 1e12:.1f} TFLOP/s), wgrad "
            f"{t_w * 1e3:.3f} ms, FP32 VALU fwd {t_v * 1e3:.2f} ms, network {t_m * 1e3:.2f} ms")
        del x, dy, x32, v
        torch.cuda.empty_cache()
    print(json.dumps(dict(kernel="conv16_mfma_kernel / conv16_wgrad_mfma_kernel",
                          peak_bf16_tflops=BF16_PEAK / 1e12, results=out)), flush=True)


def matrix(reps):
    """H, H^T and FBP at the 256^3 workloads (2048 hemisphere and 8192 sphere
    transducers) and the paper's 210x210x440 / 64x90 shape, FP32 and BF16
    storage.  Prints a markdown table."""
    import torch
    from paper_1304_2017_amd import synth
    from paper_1304_2017_amd.oat import Plan
    cfgs = [("B: 256^3, 2048 hemisphere, K 1024", lambda: synth.config_large(0)),
            ("E: 256^3, 8192 sphere, K 1024", lambda: synth.config_e(0)),
            ("P: 210x210x440 at 0.14 mm, 64x90 rings, K 1022", lambda: synth.config_p(0))]
    print("| workload | storage | H ms | H^T ms | FBP ms | H upd/s | H^T upd/s | FBP upd/s | "
          "nominal HBM % (H) | plan s | arc table GB | segment table GB |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for name, make in cfgs:
        geom, _, img = make()
        t0 = time.perf_counter()
        plan = Plan(geom, 0)         # the library's default table budget
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        st = plan.stats()
        NQ = float(geom.n_vox) * geom.n_det
        for dt, nbytes in ((torch.float32, 8), (torch.bfloat16, 4)):
            x = torch.from_numpy(np.asarray(img, dtype=np.float32)).cuda().to(dt)
            p = torch.empty(plan.data_shape, device="cuda", dtype=dt)
            a = torch.empty(plan.image_shape, device="cuda", dtype=dt)
            th = time_op(lambda: plan.project(x, out=p), reps)
            tt = time_op(lambda: plan.backproject(p, out=a), reps)
            tf = time_op(lambda: plan.fbp(p, out=a), reps)
            print(f"| {name} | {'f32' if dt == torch.float32 else 'bf16'} | {th * 1e3:.1f} | "
                  f"{tt * 1e3:.1f} | {tf * 1e3:.1f} | {NQ / th:.3e} | {NQ / tt:.3e} | {NQ / tf:.3e} | "
                  f"{100 * NQ / th * nbytes / HBM_PEAK:.1f} | {plan_s:.2f} | "
                  f"{st['arc_table_bytes'] / 1e9:.1f} | {st['segment_table_bytes'] / 1e9:.1f} |",
                  flush=True)
            del x, p, a
        plan.close()
        del plan
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--matrix", action="store_true",
                    help="time H, H^T, FBP at three workloads, FP32 and BF16 (markdown table)")
    ap.add_argument("--pls", choices=["c", "e"], default=None,
                    help="run PLS-TV at the 192^3/4096 (c) or 256^3/8192 (e) workload")
    ap.add_argument("--iters", type=int, default=30, help="PLS-TV iterations (--pls, --learned)")
    ap.add_argument("--learned", action="store_true",
                    help="train the learned preconditioner and time PLS-TV plain vs learned")
    ap.add_argument("--phantoms", type=int, default=64, help="training phantoms (--learned)")
    ap.add_argument("--epochs", type=int, default=5, help="training epochs (--learned)")
    ap.add_argument("--sph", action="store_true",
                    help="time the spherical-voxel model H_sph and H_sph^T at 64^3 / 2048 / 256")
    ap.add_argument("--paper", action="store_true",
                    help="the paper's simulation: FBP and PLS-Int RMSE vs data amount at 210x210x440")
    ap.add_argument("--cnn", action="store_true",
                    help="time the BF16 16->16 convolutions on the matrix cores at 128^3 and 256^3")
    ap.add_argument("--eir", action="store_true",
                    help="time H, H^T with a 64-tap EIR and the deconvolution + FBP at 256^3")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the operators run on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1304_2017_amd import synth
    from paper_1304_2017_amd.oat import Plan

    if args.matrix:
        matrix(max(args.steps, 3))
        return
    if args.pls:
        pls_run(args.pls, args.iters)
        return
    if args.learned:
        learned_run(args.phantoms, args.epochs, args.iters)
        return
    if args.eir:
        eir_run(max(args.steps, 3))
        return
    if args.cnn:
        cnn_run(max(args.steps, 3))
        return
    if args.paper:
        paper_run(args.iters if args.iters != 30 else 20)
        return
    if args.sph:
        sph_run(max(args.steps, 3))
        return
    dev = torch.device("cuda", 0)
    log("[bench] building 256^3 workload")
    geom, ells, img = synth.config_large(0, dtype=np.float32)
    t_plan = time.perf_counter()
    plan = Plan(geom, 0)
    plan_s = time.perf_counter() - t_plan
    st = plan.stats()
    log(f"[bench] plan {plan_s:.2f} s, arc table {st['arc_table_bytes'] / 1e9:.2f} GB, "
        f"segment table {st['segment_table_bytes'] / 1e9:.2f} GB")
    x = torch.from_numpy(img).to(dev)
    p = torch.empty(plan.data_shape, device=dev)
    a = torch.empty(plan.image_shape, device=dev)
    f = torch.empty(plan.image_shape, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.project(x, out=p)
        if ev is not None:
            ev[1].record(stream)
        plan.backproject(p, out=a)
        if ev is not None:
            ev[2].record(stream)
        plan.fbp(p, out=f)
        if ev is not None:
            ev[3].record(stream)

    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(args.steps):
        step(evs[s])
        log(f"[bench] step {s} queued")
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    t_h = np.mean([e[0].elapsed_time(e[1]) for e in evs])
    t_ht = np.mean([e[1].elapsed_time(e[2]) for e in evs])
    t_f = np.mean([e[2].elapsed_time(e[3]) for e in evs])
    N, Q = geom.n_vox, geom.n_det
    # headline: H and H^T updates over their own time (FBP only under ops)
    value = 2.0 * N * Q / ((t_h + t_ht) * 1e-3)
    pts = quad_points(geom)
    # Dominant kernel: the G or G^T brick kernel (the operator call also holds
    # one small data-side kernel, under 1% of its time).  G on the segment
    # table is srt_fwd_seg_kernel.
    g_name = "srt_fwd_seg_kernel" if st["segment_table_bytes"] > 0 else "srt_fwd_kernel"
    dom_name, dom_ms = ("srt_adj_kernel", t_ht) if t_ht >= t_h else (g_name, t_h)
    achieved = OPS_PER_POINT * pts / (dom_ms * 1e-3)
    traffic = measured_traffic(dom_name)
    roof = dict(bound="alu", kernel=dom_name, achieved=achieved, peak=VALU_PEAK,
                unit="VALU lane-op/s", frac=achieved / VALU_PEAK, traffic=traffic,
                ops_per_point=OPS_PER_POINT, points_per_launch=pts)
    # HBM, two readings: what an untiled kernel would stream per update (8 bytes
    # in FP32) at each operator's rate, and the measured bytes of the dominant
    # kernel per second of its launch.
    hbm = dict(nominal_frac_H=N * Q / (t_h * 1e-3) * 8.0 / HBM_PEAK,
               nominal_frac_HT=N * Q / (t_ht * 1e-3) * 8.0 / HBM_PEAK,
               nominal_frac=value * 8.0 / HBM_PEAK,
               measured_frac=(traffic / (dom_ms * 1e-3) / HBM_PEAK) if traffic else None)
    out = dict(metric="H/H^T voxel-view updates/s", value=value, unit="voxel-view updates/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="256^3 image (0.1 mm), 2048 transducers on a 40 mm "
                                    "hemisphere, 1024 samples at 20 MHz; step = H + H^T + FBP; "
                                    "value = 2 N Q / (t_H + t_HT)",
                           nx=256, n_det=Q, n_t=geom.n_t, storage="f32",
                           arc_table_bytes=st["arc_table_bytes"],
                           segment_table_bytes=st["segment_table_bytes"],
                           plan_build_s=plan_s),
               ops=dict(H_ms=t_h, HT_ms=t_ht, FBP_ms=t_f,
                        H_updates_per_s=N * Q / (t_h * 1e-3),
                        HT_updates_per_s=N * Q / (t_ht * 1e-3),
                        FBP_updates_per_s=N * Q / (t_f * 1e-3),
                        FBP_valu_frac=OPS_PER_FBP_UPDATE * N * Q / (t_f * 1e-3) / VALU_PEAK),
               roofline=roof, hbm=hbm)
    if not args.no_cpu:
        log("[bench] oracle CPU baseline (bounded sample)")
        p_np = p.double().cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(geom, img.astype(np.float64), p_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
