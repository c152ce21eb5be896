#!/usr/bin/env python3
"""Benchmark: k-point band solves per second on one MI355X.

Workload (one "step" = the whole hot path once): the 1132-phase Voronoi
cell on a 64 x 64 pixel grid (seeded, properties E log-U[1,200] GPa,
nu U[0.2,0.4], rho log-U[1000,8000] kg/m^3), 21 x 21 plane waves
(2N = 882 displacement unknowns), 60 k-points on Gamma-X-M-Gamma, 18 bands,
FP64 throughout:
  structure factors -> Toeplitz assembly -> Cholesky factors and the
  k-independent coefficient matrices (plan build), then for all 60 k:
  operator formation -> reduction to tridiagonal form -> tridiagonal
  eigenpairs -> back-transform -> FP64 Rayleigh-Ritz.
The cell's phase map and property table are uploaded before timing; the
frequencies are written to device memory.

Prints one JSON line.  The CPU baseline is the oracle timed on a bounded
sample of the same workload's k-points on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "k-point band solves/sec at ≤1e-5 rel freq err (mixed/batched/surrogate vs FP64)"
HBM_PEAK_GBS = 8000.0


HB = 16                 # band width of the two-stage reduction
FP64_PEAK_TFLOPS = 78.6  # vector FP64 (fp64 matrix cores have the same rate)
CMAC = 8.0               # real flops of one complex multiply-add


def _trailing(n: int):
    """(m, kq) of every stage-1 panel step of an item of order n: the trailing
    matrix after the panel has order m, the panel has kq = min(HB, m) reflectors."""
    out, c0 = [], 0
    while n - c0 - HB > 0:
        m = n - c0 - HB
        out.append((m, min(HB, m)))
        c0 += HB
    return out


def hb2st_flops(n: int) -> float:
    """Algorithmic flops of the bulge chasing of one item: per block of L rows,
    the right application of the previous reflector and the left application of
    the new one to the L x HB block below the band (2 L HB + 2 L (HB-1) complex
    MACs, none for the first block of a sweep), the Hermitian product D v and the
    rank-2 update of the block's lower triangle (L^2 + L (L+1))."""
    tot = 0
    for i in range(n - 1):
        s, k = i + 1, 0
        while s <= n - 1:
            L = min(HB, n - s)
            c = L * L + L * (L + 1) + L
            if k > 0:
                c += 2 * L * HB + 2 * L * (HB - 1)
            tot += c
            s += HB
            k += 1
    return CMAC * tot


def backtransform_flops(n: int, nb: int) -> float:
    """Applying every reflector of both stages to nb eigenvector columns:
    H z = z - tau v (v^H z) costs two complex MACs per reflector entry and column."""
    t = n - 1
    q, r = divmod(t, HB)
    n_refl = HB * q * (q + 1) // 2 + r * (q + 1)
    s2 = 2 * HB * n_refl * nb
    s1 = sum(2 * m * kq * nb + kq * kq * nb for m, kq in _trailing(n))
    return CMAC * (s2 + s1)


# Roofline models of the kernels that can dominate a step: (bound, unit, peak,
# algorithmic amount of one item of order n).  Bytes are complex FP64 entries
# moved once: the Hermitian trailing matrix is stored by its lower triangle.
def roofline_models(n: int, nb: int):
    tr = _trailing(n)
    return {
        "hb2st": ("alu", "TFLOP/s", FP64_PEAK_TFLOPS, hb2st_flops(n)),
        "he2hb_her2k": ("hbm", "GB/s", HBM_PEAK_GBS,
                        sum(16.0 * m * (m + 1) + 2 * 16.0 * m * kq for m, kq in tr)),
        "he2hb_hemm": ("hbm", "GB/s", HBM_PEAK_GBS,
                       sum(8.0 * m * (m + 1) + 2 * 16.0 * m * kq for m, kq in tr)),
        "he2hb_panel": ("hbm", "GB/s", HBM_PEAK_GBS, sum(2 * 16.0 * m * HB for m, kq in tr)),
        "backtransform": ("alu", "TFLOP/s", FP64_PEAK_TFLOPS, backtransform_flops(n, nb)),
    }


def measured_traffic(kernel: str, shape):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary of this workload, or None when it is missing, was taken on other
    sources of that kernel or on another launch shape (items per launch)."""
    from paper_1310_6380_amd.profile_summary import source_digest
    path = os.path.join(HERE, "profiles", "hbm_traffic_voronoi1132_fp64.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        text = fh.read()
    want = "launch shape: " + ",".join(str(v) for v in shape)
    if want not in text:
        return None
    with open(path) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 6 and cells[0] == kernel:
                return float(cells[4]) if cells[5] == source_digest(kernel) else None
    return None


def cpu_info():
    """CPU model, usable cores and the BLAS the oracle's LAPACK calls run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            blas.append({"api": i.get("internal_api"), "version": i.get("version"),
                         "threads": i.get("num_threads"), "library": os.path.basename(i.get("filepath", ""))})
    except Exception:
        pass
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas": blas}


def cpu_baseline(cell, M, Q, nb, omega_gpu, n_single=6):
    """The oracle on every k-point of the headline cell with all host cores
    (its LAPACK threads), and on n_single of them with one thread."""
    from oracle import mixed_oracle as mo
    from oracle.compare import band_error
    info = cpu_info()
    threads = max([b["threads"] or 1 for b in info["blas"]] or [1])
    progress("cpu baseline: oracle on all", Q.shape[0], "k-points,", threads, "threads")
    t0 = time.perf_counter()
    ref, _ = mo.bands(cell.phase, cell.props, cell.lattice, M, M, Q, nb)
    dt = time.perf_counter() - t0
    err = band_error(omega_gpu, ref)
    single = None
    try:
        from threadpoolctl import threadpool_limits
        idx = np.linspace(0, Q.shape[0] - 1, n_single).round().astype(int)
        progress("cpu baseline: oracle on", n_single, "k-points, 1 thread")
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            mo.bands(cell.phase, cell.props, cell.lattice, M, M, Q[idx], nb)
            d1 = time.perf_counter() - t1
        single = {"value": n_single / d1, "unit": "solves/s", "threads": 1,
                  "sample": f"{n_single} of the {Q.shape[0]} k-points (incl. the subdomain integrals), {d1:.1f} s"}
    except Exception as exc:   # threadpoolctl missing: report the all-core figure only
        single = {"error": str(exc)}
    return ({
        "value": Q.shape[0] / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": f"all {Q.shape[0]} k-points of the headline cell (incl. its subdomain integrals), "
                  f"NumPy/SciPy LAPACK, {dt:.1f} s",
        "cpu_model": info["cpu_model"], "host_cores": info["cores"], "blas": info["blas"],
        "single_thread": single,
    }, err, np.arange(Q.shape[0]), ref)


def batched_error(cfg, om_batch, n_k=3):
    """Oracle check of the batched workload: the two cells of the smallest and
    the two of the largest cutoff (2N = 1250), n_k points each."""
    from oracle import mixed_oracle as mo
    from oracle.compare import band_error
    by_m = sorted(range(len(cfg["cells"])), key=lambda i: cfg["cells"][i]["M"])
    order = by_m[:2] + by_m[-2:]
    kidx = np.linspace(0, cfg["Q"].shape[0] - 1, n_k).round().astype(int)
    worst = 0.0
    for i in order:
        c = cfg["cells"][i]
        ref, _ = mo.bands(c["cell"].phase, c["cell"].props, c["cell"].lattice, c["M"], c["M"],
                          cfg["Q"][kidx], cfg["n_bands"])
        worst = max(worst, band_error(om_batch[i][kidx], ref))
    return worst


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_timed(fn, steps, warmup, mvpb, name=""):
    for i in range(warmup):
        fn()
        progress(name, "warm-up step", i + 1, "of", warmup)
    mvpb.device_synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn()
        progress(name, "timed step", i + 1, "of", steps)
    mvpb.device_synchronize()
    return (time.perf_counter() - t0) / steps


def variant_mixed(mvpb, ctx, dcell, M, Q, nb, steps, warmup):
    """Same cell and k list; FP32 structure factors, FP32 reduction to
    tridiagonal form and back-transform, FP64 Rayleigh-Ritz."""
    prec = mvpb.PREC_SF_FP32 | mvpb.PREC_EIG_FP32_RR64
    out = {}

    def step():
        plan = dcell.plan(M, M, prec)
        out["om"] = plan.solve(Q, nb)
        plan.close()

    dt = run_timed(step, steps, warmup, mvpb, "mixed")
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt,
            "precision": "SF fp32 (MFMA), reduction fp32, Rayleigh-Ritz fp64"}, out["om"]


def variant_batched(mvpb, ctx, steps, warmup):
    """256 seeded two-phase inclusion cells on 32x32, cutoff M uniform in 5..12
    (2N = 242..1250), 40 k each, 10 bands, FP64: every cell's plan build and
    all 10 240 (cell, k) eigensolves in one captured graph launch per step
    (mvpb_solve_cells).  Also timed: the same work as separate calls (batched
    plan build, then the eigensolve graphs of mvpb_solve_batch)."""
    from synth import config2
    cfg = config2()
    cells = [ctx.cell(c["cell"].phase, c["cell"].props, c["cell"].lattice) for c in cfg["cells"]]
    Ms = [c["M"] for c in cfg["cells"]]
    Q, nb = cfg["Q"], cfg["n_bands"]
    out = {}

    def step():
        out["om"] = ctx.solve_cells(cells, Ms, [Q] * len(cells), nb)

    def step_calls():
        plans = ctx.plans(cells, Ms)
        out["om2"] = ctx.solve_batch(plans, [Q] * len(plans), nb)
        for p in plans:
            p.close()

    dt = run_timed(step, steps, warmup, mvpb, "batched, one graph")
    dt2 = run_timed(step_calls, 2, 1, mvpb, "batched, separate calls")
    same = all(np.array_equal(a, b) for a, b in zip(out["om"], out["om2"]))
    items = len(cells) * Q.shape[0]
    # one more plan build with every kernel timed: assembly roofline
    ctx.profile(True)
    plans = ctx.plans(cells, Ms)
    mvpb.device_synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    for p in plans:
        p.close()
    roof = assembly_roofline(mvpb, ctx, cfg, cells, prof)
    return {"value": items / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "items": items,
            "launch": "one graph per step: plan build of 256 cells and 10 240 eigensolves (mvpb_solve_cells)",
            "separate_calls": {"value": items / dt2, "ms_per_step": 1e3 * dt2,
                               "what": "mvpb_plan_create_batch, then mvpb_solve_batch", "bitwise_equal": same},
            "precision": "fp64", "assembly_roofline": roof,
            "plan_build_kernel_ms": {k: v[0] for k, v in prof.items() if v[1]}}, out["om"], cfg


def variant_hex_polygons(mvpb, ctx, steps, warmup):
    """Steel cylinders (d = 4 mm) in epoxy on the hexagonal lattice
    (a = 6.023 mm), the example of Sec. 5, given as polygons (the cell
    parallelogram, a 256-gon of the disk's area and its clockwise hole):
    21x21 plane waves (2N = 882), 60 k on X-Gamma-J-X, 12 bands, FP64.  Also
    reports the complete stop bands over the path."""
    from synth import hex_steel_epoxy, kpath_xgjx
    c = hex_steel_epoxy(256)
    dcell = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice)
    M, nb = 10, 12
    Q = kpath_xgjx(60)
    out = {}

    def step():
        plan = dcell.plan(M)
        out["om"] = plan.solve(Q, nb)
        plan.close()

    dt = run_timed(step, steps, warmup, mvpb, "hex polygons")
    f = out["om"] / (2.0 * np.pi) / 1e3
    gaps = [[round(float(f[:, b].max()), 1), round(float(f[:, b + 1].min()), 1)]
            for b in range(nb - 1) if f[:, b + 1].min() - f[:, b].max() >= 10.0]
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "precision": "fp64",
            "two_N": 2 * (2 * M + 1) ** 2, "k_points": int(Q.shape[0]), "n_bands": nb,
            "stop_bands_khz": gaps, "paper_stop_bands_khz_at_M5": [[120, 262], [427, 473]]}, out["om"], (c, M, Q, nb)


def variant_hex_1132(mvpb, ctx, steps, warmup):
    """The 1132-element hexagonal cell of Sec. 5 (elements of steel's stiffness,
    density 10^6 x centroid height), as 1132 polygons: 21x21 plane waves
    (2N = 882), 60 k on X-Gamma-J-X, 18 bands, FP64."""
    from synth import hex_graded_1132, kpath_xgjx
    c = hex_graded_1132()
    dcell = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice)
    M, nb = 10, 18
    Q = kpath_xgjx(60)
    out = {}

    def step():
        plan = dcell.plan(M)
        out["om"] = plan.solve(Q, nb)
        plan.close()

    dt = run_timed(step, steps, warmup, mvpb, "hex 1132 elements")
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "precision": "fp64",
            "two_N": 2 * (2 * M + 1) ** 2, "k_points": int(Q.shape[0]), "n_bands": nb,
            "polygons": len(c.polygons)}, out["om"], (c, M, Q, nb)


def variant_stress(mvpb, ctx, dcell, M, Q, nb, steps, warmup):
    """Same cell and k list as the headline, FP64, with the displacement modes
    U and the stress modes S = -Phi^-1 H* U returned to the host."""
    out = {}

    def step():
        plan = dcell.plan(M)
        om, U = plan.solve(Q, nb, vectors=True)
        out["om"], out["U"], out["S"] = om, U, plan.stress(Q, U)
        plan.close()

    dt = run_timed(step, steps, warmup, mvpb, "stress modes")
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "precision": "fp64",
            "outputs": "omega, U (2N per band), S (3N per band), host"}, out


def variant_surrogate(mvpb, ctx, n_train=8192, n_test=1024, epochs=60, label_chunk=512):
    """Binary GRF cells on 32x32 (correlation length 4 px, fill U[0.2,0.8]),
    labels by the batched FP64 solver at 15x15 plane waves, 40 k, 10 bands;
    network trained by the library's kernels (BF16 matrix cores) on the
    standardised labels (cosine step-size decay); held-out error on cells it
    has not seen; inference timed on batches of 4096 cells; what it gains:
    the best verified gap among its 32 top-ranked held-out cells against 32
    random ones (same number of plain solves), and a screening loop with
    plain-solve verification and fallback.  One "solve" = one cell at one k."""
    from paper_1310_6380_amd import screening as sc
    from synth import config4_cells
    cells = config4_cells(0, n_train + n_test)
    t0 = time.perf_counter()
    y = sc.label_cells(ctx, cells, chunk=label_chunk)
    t_label = time.perf_counter() - t0
    progress("surrogate labels", cells.shape[0], "cells in", round(t_label, 1), "s")
    norm = sc.Normalizer(y[:n_train])
    net = mvpb.Surrogate(ctx, max_batch=4096, precision=1, seed=0)
    t0 = time.perf_counter()
    losses = sc.train(net, cells[:n_train], y[:n_train], epochs=epochs, batch=256, lr=2e-3, lr_end=2e-5,
                      log=progress, norm=norm)
    t_train = time.perf_counter() - t0
    pred = sc.predict(net, cells[n_train:], norm)
    err = sc.relative_errors(pred, y[n_train:])
    ref = y[n_train:].reshape(-1, sc.N_K, sc.N_BANDS)
    rel_top = np.abs(pred.reshape(ref.shape) - ref) / ref[:, :, -1:]
    # gain at an equal budget of plain solves (32 cells verified each)
    b, budget = 2, 32
    tg = sc.band_gap(y[n_train:], b)
    pick = np.argsort(-sc.band_gap(pred, b))[:budget]
    rng = np.random.default_rng(0)
    draws = np.stack([rng.choice(tg.size, budget, replace=False) for _ in range(400)])
    best_r = tg[draws].max(axis=1)
    frac = float(np.mean(tg >= tg[pick].max()))
    batch = np.resize(cells[n_train:], (4096, 32, 32))
    dcells = mvpb.DeviceBuffer(batch.size).upload(batch)
    dout = mvpb.DeviceBuffer(4 * 4096 * 400)

    def step():
        net.infer_device(4096, dcells.value, dout.value)

    dt = run_timed(step, 5, 2, mvpb, "surrogate inference")
    stats = sc.screen(ctx, net, cells[:64], b=b, rounds=2, n_candidates=4096, top_k=16, log=progress, norm=norm)
    net.close()
    return {"value": 4096 * sc.N_K / dt, "unit": "solves/s", "cells_per_s": 4096 / dt,
            "ms_per_batch_4096": 1e3 * dt, "precision": "bf16 matrix cores, fp32 accumulate",
            "held_out_rel_err": {"p50": float(np.median(err)), "p99": float(np.percentile(err, 99)),
                                 "max": float(err.max()), "cells": int(n_test),
                                 "definition": "per cell, worst relative error over its 400 outputs",
                                 "median_rel_to_top_band": float(np.median(rel_top))},
            "train": {"cells": n_train, "epochs": epochs, "seconds": t_train, "final_loss": float(losses[-1]),
                      "cells_per_s": n_train * epochs / t_train},
            "labels": {"cells": int(cells.shape[0]), "solves_per_s": cells.shape[0] * sc.N_K / t_label},
            "gain_equal_budget": {"band_pair": [b, b + 1], "budget_cells": budget,
                                  "surrogate_best_gap": float(tg[pick].max()),
                                  "surrogate_mean_gap": float(tg[pick].mean()),
                                  "random_best_gap_p50": float(np.median(best_r)),
                                  "random_best_gap_p90": float(np.percentile(best_r, 90)),
                                  "random_solves_to_reach_surrogate_best": float(sc.N_K / max(frac, 1e-9))},
            "screening": {"candidates": stats["predicted"], "verified": stats["verified"],
                          "fallback_rate": stats["fallbacks"] / max(1, stats["verified"]),
                          "best_verified_gap_b2_b3": stats["best_gap"],
                          "rounds": stats["rounds"],
                          "surrogate_s_per_cell": stats["t_surrogate"] / stats["predicted"],
                          "solve_s_per_cell": stats["t_solve"] / stats["verified"]}}


def run_median(fn, steps, warmup, mvpb, name=""):
    """Median of `steps` individually timed steps (device drained around
    each) after `warmup` untimed ones."""
    for _ in range(warmup):
        fn()
    mvpb.device_synchronize()
    ts = []
    for i in range(steps):
        t0 = time.perf_counter()
        fn()
        mvpb.device_synchronize()
        ts.append(time.perf_counter() - t0)
    progress(name, "median of", steps, "steps:", round(1e3 * float(np.median(ts)), 2), "ms")
    return float(np.median(ts))


def variant_precision(mvpb, ctx):
    """4096 Voronoi phases on 128x128, 31x31 plane waves (2N = 1922), 60 k,
    24 bands: structure factors in FP64, FP32, BF16 and split BF16, and the
    FP32 reduction with FP64 Rayleigh-Ritz (alone and with split-BF16 or
    FP32 structure factors).  3 warm-up steps, median of 5."""
    from synth import config3
    cfg = config3()
    cell, M, Q, nb = cfg["cell"], cfg["M"], cfg["Q"], cfg["n_bands"]
    dcell = ctx.cell(cell.phase, cell.props, cell.lattice)
    res, oms = {}, {}
    for name, prec in (("fp64", mvpb.PREC_FP64), ("sf_fp32", mvpb.PREC_SF_FP32), ("sf_bf16", mvpb.PREC_SF_BF16),
                       ("sf_bf16x3", mvpb.PREC_SF_BF16X3), ("eig_fp32_rr64", mvpb.PREC_EIG_FP32_RR64),
                       ("sf_fp32_eig_fp32_rr64", mvpb.PREC_SF_FP32 | mvpb.PREC_EIG_FP32_RR64),
                       ("sf_bf16x3_eig_fp32_rr64", mvpb.PREC_SF_BF16X3 | mvpb.PREC_EIG_FP32_RR64)):
        out = {}

        def step():
            plan = dcell.plan(M, M, prec)
            out["om"] = plan.solve(Q, nb)
            plan.close()

        ctx.set_accuracy(0.0)   # every variant is timed and reported, whatever its estimate
        try:
            dt = run_median(step, 5, 3, mvpb, "precision " + name)
        finally:
            ctx.set_accuracy(1e-5)
        res[name] = {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt,
                     "offered_as_mixed_path": name != "sf_bf16"}
        if prec & mvpb.PREC_EIG_FP32_RR64:
            res[name]["estimated_rel_freq_err"] = ctx.last_accuracy()
        oms[name] = out["om"]
    return res, oms, cfg


def variant_simple_cell(mvpb, ctx, steps=20, warmup=3):
    """The simple inclusion cell: circle r = 0.3a on 16x16 pixels (E 70 GPa,
    nu 0.33, rho 2700 in E 3.5 GPa, nu 0.35, rho 1180), 7x7 plane waves
    (2N = 98), 30 k on Gamma-X-M-Gamma, 6 bands, FP64; plan build + solve per
    step, median of 20."""
    from synth import config0
    c = config0()
    cell, M, Q, nb = c["cell"], c["M"], c["Q"], c["n_bands"]
    dcell = ctx.cell(cell.phase, cell.props, cell.lattice)
    om_dev = mvpb.DeviceBuffer(8 * Q.shape[0] * nb)

    def step():
        plan = dcell.plan(M)
        plan.solve_device(Q, nb, om_dev.value)
        plan.close()

    dt = run_median(step, steps, warmup, mvpb, "simple cell")
    om = om_dev.to_numpy(np.float64, (Q.shape[0], nb))
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "precision": "fp64",
            "two_N": 2 * (2 * M + 1) ** 2, "k_points": int(Q.shape[0]), "n_bands": nb,
            "timing": "median of %d steps after %d warm-ups" % (steps, warmup)}, om, c


def variant_anisotropic(mvpb, ctx, steps=5, warmup=2):
    """General layout: the 1132-phase Voronoi map of the headline with a
    random full engineering-Voigt compliance per phase (shear-normal coupling
    non-zero, seeded), 21x21 plane waves (2N = 882, full 3N x 3N Phi
    factored), 60 k, 18 bands, FP64."""
    from synth import config1, random_voigt_props, rng_for
    c = config1()
    rows = random_voigt_props(c["cell"].n_phases, rng_for(101, 0))
    dcell = ctx.cell(c["cell"].phase, rows)
    M, Q, nb = c["M"], c["Q"], c["n_bands"]
    out = {}

    def step():
        plan = dcell.plan(M)
        out["om"] = plan.solve(Q, nb)
        plan.close()

    dt = run_median(step, steps, warmup, mvpb, "anisotropic")
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "precision": "fp64",
            "two_N": 2 * (2 * M + 1) ** 2, "k_points": int(Q.shape[0]), "n_bands": nb}, out["om"], (c, rows)


def kpath_cubic(n_k):
    """n_k points equally spaced in arc length on Gamma-X-M-Gamma-R of a cubic
    lattice (fractional: X = (1/2,0,0), M = (1/2,1/2,0), R = (1/2,1/2,1/2))."""
    pts = np.array([[0, 0, 0], [0.5, 0, 0], [0.5, 0.5, 0], [0, 0, 0], [0.5, 0.5, 0.5]], dtype=np.float64)
    seg = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    s = np.linspace(0.0, seg.sum(), n_k)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    out = []
    for t in s:
        k = min(np.searchsorted(cum, t, side="right") - 1, len(seg) - 1)
        f = (t - cum[k]) / seg[k]
        out.append(pts[k] + f * (pts[k + 1] - pts[k]))
    return np.array(out)


def sphere_voxels(n, r=0.3):
    x = (np.arange(n) + 0.5) / n - 0.5
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    return (X ** 2 + Y ** 2 + Z ** 2 <= r * r).astype(np.int32)


def variant_voxels(mvpb, ctx, steps=5, warmup=2):
    """Three-dimensional cell: a sphere r = 0.3a of the inclusion material in
    the matrix of the simple cell, 16^3 voxels, 7^3 plane waves (3N = 1029
    displacement, 6N = 2058 stress unknowns), 30 k on Gamma-X-M-Gamma-R,
    12 bands, FP64."""
    from synth import INCLUSION_PROPS, MATRIX_PROPS
    phase = sphere_voxels(16)
    props = np.array([MATRIX_PROPS, INCLUSION_PROPS])
    dcell = ctx.cell_voxels(phase, props)
    M, nb = 3, 12
    Q = kpath_cubic(30)
    out = {}

    def step():
        plan = dcell.plan(M)
        out["om"] = plan.solve(Q, nb)
        plan.close()

    dt = run_median(step, steps, warmup, mvpb, "voxels")
    return {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "precision": "fp64",
            "three_N": 3 * (2 * M + 1) ** 3, "k_points": int(Q.shape[0]), "n_bands": nb}, out["om"], (phase, props, M, Q, nb)


def variant_sensitivities(mvpb, ctx, dcell, M, Q, nb, steps=3, warmup=1):
    """d lambda / d w_f of every pixel of the headline cell (7 fields x 4096
    pixels) for every band and k of the headline workload, returned to the
    host; timed after the solve that supplies omega and U."""
    plan = dcell.plan(M)
    om, U = plan.solve(Q, nb, vectors=True)

    def step():
        plan.sensitivities(Q, om, U, (64, 64))

    dt = run_median(step, steps, warmup, mvpb, "sensitivities")
    plan.close()
    items = Q.shape[0] * nb
    return {"value": items / dt, "unit": "(k, band) gradients/s", "ms_per_step": 1e3 * dt,
            "outputs_per_item": 7 * 64 * 64, "items": items, "precision": "fp64"}


def variant_optimisation(mvpb, ctx, iters=10):
    """Gradient-based band-gap design: a seeded GRF 32x32 start, per-pixel
    material fraction between the two materials of the simple cell, 15x15
    plane waves, 40 k on Gamma-X-M-Gamma, gap between bands 3 and 4; every
    step verified by a plain FP64 solve."""
    from paper_1310_6380_amd.optimize import Design
    from synth import INCLUSION_PROPS, MATRIX_PROPS, config4_cells
    d = Design(ctx, MATRIX_PROPS, INCLUSION_PROPS, M=7, Q=mvpb.kpath_square(40), b=2)
    x0 = config4_cells(0, 1)[0].astype(np.float64)
    t0 = time.perf_counter()
    x, hist = d.optimise(x0, iters=iters, log=progress)
    dt = time.perf_counter() - t0
    return {"iterations": iters, "gap_start": float(hist[0]), "gap_end": float(hist[-1]),
            "accepted_steps": len(hist) - 1, "plain_solves": d.solves, "seconds": dt,
            "solves_per_s": d.solves / dt}


def assembly_roofline(mvpb, ctx, cfg, cells_dev, prof):
    """Roofline of the batched plan build's assembly kernels from the kernel
    timers of one step: the Toeplitz scatter against HBM (algorithmic bytes:
    the 3 N x N complex blocks written per cell) and the structure factors
    against the FP64 matrix-core peak (algorithmic flops of the two
    contractions per cell: 4 fields x (4 nx ny nq + 8 nm nq nx) real flops)."""
    w_bytes = 0.0
    sf_flops = 0.0
    for c in cfg["cells"]:
        M, nx, ny = c["M"], c["cell"].nx, c["cell"].ny
        N = (2 * M + 1) ** 2
        nm = nq = 4 * M + 1
        w_bytes += 3.0 * N * N * 16.0
        sf_flops += 4.0 * (4.0 * nx * ny * nq + 8.0 * nm * nq * nx)
    out = {}
    t_sc, n_sc = prof.get("toeplitz_scatter", (0.0, 0))
    if n_sc:
        ach = w_bytes / (t_sc / 1e3) / 1e9
        out["toeplitz_scatter"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": ach / HBM_PEAK_GBS, "launches": n_sc, "ms": t_sc,
                                   "algorithmic_bytes": w_bytes}
    t_sf, n_sf = prof.get("structure_factors", (0.0, 0))
    if n_sf:
        ach = sf_flops / (t_sf / 1e3) / 1e12
        out["structure_factors"] = {"bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": ach / FP64_PEAK_TFLOPS, "launches": n_sf, "ms": t_sf,
                                    "algorithmic_flops": sf_flops}
    return out


PAPER_NUMBERS = [
    {"what": "1132-element hexagonal cell (one phase per element), 18 branches", "time": "18.5 s (abstract: under 20 s)",
     "k_points": "not stated; 70 assumed", "derived_solves_per_s": 70 / 18.5, "plane_waves": "M = 3 (2N = 98)",
     "hardware": "NVIDIA Quadro K2000 (Kepler, 384 CUDA cores, 2 GB) in a desktop, Python + CUDA; precision not stated",
     "compare_with": "variants.hex_1132_element_polygons (2N = 882)"},
    {"what": "first branches of a simpler cell", "time": "about 2 s (abstract: under 2.5 s)", "k_points": "70",
     "derived_solves_per_s": 70 / 2.5, "plane_waves": "small M (about 2)",
     "hardware": "NVIDIA Quadro K2000, desktop; precision not stated",
     "compare_with": "variants.simple_cell (2N = 98)"},
    {"what": "full band structure, 18 branches, 1000 elements", "time": "90 s", "k_points": "70",
     "derived_solves_per_s": 70 / 90.0, "plane_waves": "M = 5 (2N = 242)",
     "hardware": "NVIDIA Quadro K2000, desktop; precision not stated", "compare_with": "value (2N = 882)"},
]


def copy_calibration(mib: int):
    """One copy of a known byte count by the library's copy16 kernel, so that
    hardware traffic counters can be scaled to bytes."""
    from paper_1310_6380_amd import mvpb
    nbytes = mib << 20
    ctx = mvpb.Context(0)
    src, dst = mvpb.DeviceBuffer(nbytes), mvpb.DeviceBuffer(nbytes)
    src.upload(np.arange(nbytes // 8, dtype=np.int64))
    t0 = time.perf_counter()
    ctx.copy_device(dst.value, src.value, nbytes)
    dt = time.perf_counter() - t0
    ok = bool(np.array_equal(dst.to_numpy(np.int64, (nbytes // 8,))[-4:], np.arange(nbytes // 8 - 4, nbytes // 8)))
    print(json.dumps({"copy_bytes": nbytes, "read_bytes": nbytes, "write_bytes": nbytes, "seconds": dt,
                      "tail_ok": ok}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=6,
                    help="k-points timed on the CPU oracle with one thread (0 = skip the CPU baseline)")
    ap.add_argument("--surrogate-full", action="store_true",
                    help="only the surrogate study at full scale: 50 000 GRF cells, 45 000 trained, 5 000 held out")
    ap.add_argument("--surrogate-kernels", action="store_true",
                    help="only the surrogate's kernels (for profiling): 30 training steps of 256 seeded GRF cells "
                         "and 5 inference batches of 4096")
    ap.add_argument("--shape", default="",
                    help="fixed launch shape 'parts,group,workgroups' of the headline instead of autotuning it")
    ap.add_argument("--assembly", action="store_true",
                    help="only the batched plan build of the 256-cell inclusion workload, twice (for profiling)")
    ap.add_argument("--no-variants", action="store_true", help="only the headline FP64 workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB once with the library's plain copy kernel (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.surrogate_kernels:
        from paper_1310_6380_amd import mvpb
        from synth import config4_cells
        ctx = mvpb.Context(0)
        net = mvpb.Surrogate(ctx, max_batch=4096, precision=1, seed=0)
        cells = config4_cells(0, 4096)
        y = np.random.default_rng(0).uniform(0.1, 1.0, (4096, 400)).astype(np.float32)
        dc = mvpb.DeviceBuffer(cells.size).upload(cells)
        dy = mvpb.DeviceBuffer(y.nbytes).upload(y)
        dout = mvpb.DeviceBuffer(y.nbytes)
        t0 = time.perf_counter()
        for i in range(30):
            net.train_step_device(256, dc.value + 1024 * 256 * (i % 16), dy.value + 4 * 400 * 256 * (i % 16))
        mvpb.device_synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            net.infer_device(4096, dc.value, dout.value)
        mvpb.device_synchronize()
        t2 = time.perf_counter()
        print(json.dumps({"surrogate_kernels": {"train_ms_per_step_256": 1e3 * (t1 - t0) / 30,
                                                "infer_ms_per_batch_4096": 1e3 * (t2 - t1) / 5}}), flush=True)
        net.close()
        ctx.close()
        return
    if args.assembly:
        from paper_1310_6380_amd import mvpb
        from synth import config2
        ctx = mvpb.Context(0)
        cfg = config2()
        cells = [ctx.cell(c["cell"].phase, c["cell"].props, c["cell"].lattice) for c in cfg["cells"]]
        Ms = [c["M"] for c in cfg["cells"]]
        for step in range(2):
            plans = ctx.plans(cells, Ms)
            mvpb.device_synchronize()
            for p in plans:
                p.close()
            progress("assembly step", step + 1)
        ctx.close()
        return
    if args.surrogate_full:
        from paper_1310_6380_amd import mvpb
        ctx = mvpb.Context(0)
        res = variant_surrogate(mvpb, ctx, n_train=45000, n_test=5000, epochs=60, label_chunk=1024)
        print(json.dumps({"surrogate_grf_cells_full": res}), flush=True)
        ctx.close()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note",
              file=sys.stderr)
        sys.exit(2)

    from paper_1310_6380_amd import mvpb
    from synth import config1

    cfg = config1()
    cell, M, Q, nb = cfg["cell"], cfg["M"], cfg["Q"], cfg["n_bands"]
    n = 2 * (2 * M + 1) ** 2
    ctx = mvpb.Context(0)
    dcell = ctx.cell(cell.phase, cell.props, cell.lattice)

    om_dev = mvpb.DeviceBuffer(8 * Q.shape[0] * nb)   # outputs stay in HBM

    # launch shape of the eigensolve for this operator size, by the library's autotuner
    # (or fixed with --shape, e.g. to profile the shape a bench run chose)
    tune_ms, tune_entry = None, []
    if args.shape:
        parts, group, wg = (int(v) for v in args.shape.split(","))
        ctx.set_launch_shape(n, parts, group, wg)
    else:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            cache = os.path.join(td, "tuning.json")
            tplan = dcell.plan(M)
            tune_ms = tplan.autotune(Q, nb, cache)
            tplan.close()
            with open(cache) as fh:
                tune_entry = [json.loads(line.strip().rstrip(",")) for line in fh if '"device"' in line]
    shape = ctx.launch_shape(n)
    progress("launch shape (parts, group, workgroups):", shape, tune_entry)

    def step():
        plan = dcell.plan(M)
        plan.solve_device(Q, nb, om_dev.value)
        plan.close()

    for i in range(args.warmup):
        step()
        progress("fp64 warm-up step", i + 1)
    mvpb.device_synchronize()
    # per-kernel breakdown: every launch bracketed by HIP events (untimed pass;
    # the events add about 5 % to a step)
    ctx.profile(True)
    for i in range(args.steps):
        step()
    mvpb.device_synchronize()
    prof_all = ctx.profile_read()
    progress("per-kernel pass done")
    dom_name = max(prof_all.items(), key=lambda kv: kv[1][0])[0]
    # timed steps: only the dominant kernel family is bracketed by events
    ctx.profile_only([dom_name])
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        progress("fp64 timed step", i + 1)
    mvpb.device_synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_step = 1e3 * dt / args.steps
    value = Q.shape[0] * args.steps / dt

    # roofline of the dominant kernel: algorithmic work per launch over the
    # kernel's average launch time (HIP events on the context stream)
    name = dom_name
    tot_ms, launches = prof[name]
    models = roofline_models(n, nb)
    roof = {"kernel": name, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": tot_ms / max(launches, 1), "launches": launches}
    if name in models and launches:
        bound, unit, peak, per_item = models[name]
        per_launch = per_item * Q.shape[0] * args.steps / launches
        avg_s = tot_ms / launches / 1e3
        scale = 1e9 if unit == "GB/s" else 1e12
        achieved = per_launch / avg_s / scale
        roof.update({"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                     "algorithmic_per_launch": per_launch,
                     "algorithmic_unit": "bytes" if unit == "GB/s" else "flops",
                     "traffic": measured_traffic(name, shape)})
    omega = om_dev.to_numpy(np.float64, (Q.shape[0], nb))
    variants = {}
    om_mixed = om_batch = cfg2 = om_prec = cfg3 = om_hex = hexcfg = om_h1132 = h1132cfg = stress_out = None
    om_c0 = c0cfg = om_an = ancfg = om_vox = voxcfg = None
    if not args.no_variants:
        variants["simple_cell"], om_c0, c0cfg = variant_simple_cell(mvpb, ctx)
        ctx.set_accuracy(0.0)
        try:
            variants["mixed_1132_phase"], om_mixed = variant_mixed(mvpb, ctx, dcell, M, Q, nb, args.steps,
                                                                   args.warmup)
            variants["mixed_1132_phase"]["estimated_rel_freq_err"] = ctx.last_accuracy()
        finally:
            ctx.set_accuracy(1e-5)
        variants["stress_modes_1132_phase"], stress_out = variant_stress(mvpb, ctx, dcell, M, Q, nb,
                                                                        max(1, args.steps // 2), 1)
        variants["batched_256_cells"], om_batch, cfg2 = variant_batched(mvpb, ctx, max(1, args.steps // 2), 1)
        variants["surrogate_grf_cells"] = variant_surrogate(mvpb, ctx)
        variants["precision_4096_phase"], om_prec, cfg3 = variant_precision(mvpb, ctx)
        variants["hex_steel_epoxy_polygons"], om_hex, hexcfg = variant_hex_polygons(mvpb, ctx, args.steps,
                                                                                    args.warmup)
        variants["hex_1132_element_polygons"], om_h1132, h1132cfg = variant_hex_1132(mvpb, ctx, args.steps,
                                                                                     args.warmup)
        variants["anisotropic_1132_phase"], om_an, ancfg = variant_anisotropic(mvpb, ctx)
        variants["voxel_sphere_3d"], om_vox, voxcfg = variant_voxels(mvpb, ctx)
        variants["sensitivities_1132_phase"] = variant_sensitivities(mvpb, ctx, dcell, M, Q, nb)
        variants["gradient_band_gap_design"] = variant_optimisation(mvpb, ctx)
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Voronoi cell)",
        "config": {"workload": "1132-phase Voronoi cell, 64x64 pixels, 21x21 plane waves (2N=882), "
                               "60 k on G-X-M-G, 18 bands, FP64",
                   "k_points": int(Q.shape[0]), "n_bands": nb, "two_N": n},
        "roofline": roof,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof_all.items() if v[1]},
        "paper_reference": PAPER_NUMBERS,
        "autotune": {"ms_per_solve_call": tune_ms, "entries": tune_entry, "launch_shape": list(shape)},
    }
    if variants:
        out["variants"] = variants
    if args.cpu_sample > 0:
        cb, err, ref_idx, ref = cpu_baseline(cell, M, Q, nb, omega, args.cpu_sample)
        out["cpu_baseline"] = cb
        out["max_rel_freq_err_vs_oracle"] = err
        if om_mixed is not None:
            from oracle.compare import band_error
            variants["mixed_1132_phase"]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om_mixed[ref_idx], ref)
        if om_c0 is not None:
            from oracle import mixed_oracle as mo
            from oracle.compare import band_error
            c0 = c0cfg["cell"]
            t0 = time.perf_counter()
            ref0, _ = mo.bands(c0.phase, c0.props, c0.lattice, c0cfg["M"], c0cfg["M"], c0cfg["Q"], c0cfg["n_bands"])
            d0 = time.perf_counter() - t0
            variants["simple_cell"]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om_c0, ref0)
            variants["simple_cell"]["cpu_oracle"] = {"value": c0cfg["Q"].shape[0] / d0, "unit": "solves/s",
                                                     "sample": "all 30 k-points", "cores": cb["cores"]}
        if om_an is not None:
            from oracle import mixed_oracle as mo
            from oracle.compare import band_error
            from synth import voigt_rows_to_matrices
            c1, rows = ancfg
            W, rho = voigt_rows_to_matrices(rows, 2)
            props = np.stack([np.ones(len(rho)), np.zeros(len(rho)), rho], axis=1)
            kk = [3, 40]
            progress("cpu baseline: anisotropic oracle on", len(kk), "k-points")
            I = mo.subdomain_integral_tables(c1["cell"].phase, len(rho), c1["cell"].lattice, M, M)
            tabs = mo.phase_sum_tables(I, props, phase_weights=W)
            refa = np.array([mo.solve_k(mo.assemble(I, props, c1["cell"].lattice, M, M, Q[t], tables=tabs), nb)[0]
                             for t in kk])
            variants["anisotropic_1132_phase"]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om_an[kk], refa)
        if om_vox is not None:
            from oracle import mixed3d_oracle as m3
            from oracle.compare import band_error
            phase3, props3, M3, Q3, nb3 = voxcfg
            kk = [0, 11, 23]
            progress("cpu baseline: three-dimensional oracle on", len(kk), "k-points")
            refv, _ = m3.bands3(phase3, props3, np.eye(3), M3, M3, M3, Q3[kk], nb3)
            variants["voxel_sphere_3d"]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om_vox[kk], refv)
        if om_batch is not None:
            variants["batched_256_cells"]["max_rel_freq_err_vs_fp64_oracle"] = batched_error(cfg2, om_batch)
        if om_prec is not None:
            from oracle import mixed_oracle as mo
            from oracle.compare import band_error
            c3 = cfg3["cell"]
            kk = [7, 41]
            progress("cpu baseline: oracle on the 4096-phase cell,", len(kk), "k-points")
            ref3, _ = mo.bands(c3.phase, c3.props, c3.lattice, cfg3["M"], cfg3["M"], cfg3["Q"][kk], cfg3["n_bands"])
            for name, om in om_prec.items():
                variants["precision_4096_phase"][name]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om[kk], ref3)
        if stress_out is not None:
            from oracle import mixed_oracle as mo
            kk = [5, 30]
            progress("cpu baseline: oracle stress modes on", len(kk), "k-points")
            I = mo.subdomain_integral_tables(cell.phase, cell.n_phases, cell.lattice, M, M)
            tabs = mo.phase_sum_tables(I, cell.props)
            worst = 0.0
            for t in kk:
                mats = mo.assemble(I, cell.props, cell.lattice, M, M, Q[t], tables=tabs)
                ref = mo.stress_vector(mats, stress_out["U"][t].T)
                worst = max(worst, float(np.max(np.abs(stress_out["S"][t].T - ref)) / np.max(np.abs(ref))))
            variants["stress_modes_1132_phase"]["max_rel_stress_err_vs_fp64_oracle"] = worst
        if om_hex is not None:
            from oracle import mixed_oracle as mo
            from oracle.compare import band_error
            hc, hM, hQ, hnb = hexcfg
            kk = [0, 17, 41]
            progress("cpu baseline: oracle on the hexagonal polygon cell,", len(kk), "k-points")
            I = mo.polygon_integral_tables(hc.polygons, hc.poly_phase, hc.n_phases, hc.lattice, hM, hM)
            refh, _ = mo.bands(None, hc.props, hc.lattice, hM, hM, hQ[kk], hnb, I_p=I)
            variants["hex_steel_epoxy_polygons"]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om_hex[kk], refh)
        if om_h1132 is not None:
            from oracle import mixed_oracle as mo
            from oracle.compare import band_error
            hc, hM, hQ, hnb = h1132cfg
            kk = [9, 33]
            progress("cpu baseline: oracle on the 1132-element hexagonal cell,", len(kk), "k-points")
            I = mo.polygon_integral_tables(hc.polygons, hc.poly_phase, hc.n_phases, hc.lattice, hM, hM)
            refh, _ = mo.bands(None, hc.props, hc.lattice, hM, hM, hQ[kk], hnb, I_p=I)
            variants["hex_1132_element_polygons"]["max_rel_freq_err_vs_fp64_oracle"] = band_error(om_h1132[kk], refh)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
