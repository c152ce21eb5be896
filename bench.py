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


def hetrd_panel_bytes(n: int, panel: int = 32):
    """Algorithmic HBM bytes of each launch of the panel kernel for one item of
    order n: every column j of the panel multiplies the full trailing matrix
    (order n-j-1, complex FP64) by a vector once."""
    out = []
    for p in range(0, n - 1, panel):
        nbp = min(panel, n - 1 - p)
        out.append(sum(16.0 * (n - j - 1) ** 2 for j in range(p, p + nbp)))
    return out


def cpu_baseline(cell, M, Q, nb, omega_gpu, n_sample):
    from oracle import mixed_oracle as mo
    from oracle.compare import band_error
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    idx = np.linspace(0, Q.shape[0] - 1, n_sample).round().astype(int)
    progress("cpu baseline: oracle on", n_sample, "k-points")
    t0 = time.perf_counter()
    ref, _ = mo.bands(cell.phase, cell.props, cell.lattice, M, M, Q[idx], nb)
    dt = time.perf_counter() - t0
    err = band_error(omega_gpu[idx], ref)
    return ({
        "value": n_sample / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{n_sample} of the {Q.shape[0]} k-points of the same cell (incl. its subdomain integrals), "
                  f"NumPy/SciPy LAPACK, {dt:.1f} s",
    }, err, idx, ref)


def batched_error(cfg, om_batch, n_cells=4, n_k=3):
    """Oracle check of a few (small-cutoff) cells of the batched workload."""
    from oracle import mixed_oracle as mo
    from oracle.compare import band_error
    order = sorted(range(len(cfg["cells"])), key=lambda i: cfg["cells"][i]["M"])[:n_cells]
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
    (2N = 242..1250), 40 k each, 10 bands, FP64: batched per-cell assembly and
    all 10 240 (cell, k) items through one captured launch sequence per size class."""
    from synth import config2
    cfg = config2()
    cells = [ctx.cell(c["cell"].phase, c["cell"].props, c["cell"].lattice) for c in cfg["cells"]]
    Ms = [c["M"] for c in cfg["cells"]]
    Q, nb = cfg["Q"], cfg["n_bands"]
    out = {}

    def step():
        plans = ctx.plans(cells, Ms)
        out["om"] = ctx.solve_batch(plans, [Q] * len(plans), nb)
        for p in plans:
            p.close()

    dt = run_timed(step, steps, warmup, mvpb, "batched")
    items = len(cells) * Q.shape[0]
    return {"value": items / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt, "items": items,
            "precision": "fp64"}, out["om"], cfg


def variant_surrogate(mvpb, ctx, n_train=1024, n_test=256, epochs=15):
    """Binary GRF cells on 32x32 (correlation length 4 px, fill U[0.2,0.8]),
    labels by the batched FP64 solver at 15x15 plane waves, 40 k, 10 bands;
    network trained by the library's kernels (BF16 matrix cores); inference
    timed on batches of 4096 cells.  One "solve" = one cell at one k."""
    from paper_1310_6380_amd import screening as sc
    from synth import config4_cells
    cells = config4_cells(0, n_train + n_test)
    t0 = time.perf_counter()
    y = sc.label_cells(ctx, cells)
    t_label = time.perf_counter() - t0
    progress("surrogate labels", cells.shape[0], "cells in", round(t_label, 1), "s")
    net = mvpb.Surrogate(ctx, max_batch=4096, precision=1, seed=0)
    t0 = time.perf_counter()
    sc.train(net, cells[:n_train], y[:n_train], epochs=epochs, batch=256, lr=1e-3, log=progress)
    t_train = time.perf_counter() - t0
    err = sc.relative_errors(net.infer(cells[n_train:]), y[n_train:])
    batch = np.resize(cells[n_train:], (4096, 32, 32))
    dcells = mvpb.DeviceBuffer(batch.size).upload(batch)
    dout = mvpb.DeviceBuffer(4 * 4096 * 400)

    def step():
        net.infer_device(4096, dcells.value, dout.value)

    dt = run_timed(step, 5, 2, mvpb, "surrogate inference")
    stats = sc.screen(ctx, net, cells[:64], b=2, rounds=2, n_candidates=4096, top_k=16, log=progress)
    net.close()
    return {"value": 4096 * sc.N_K / dt, "unit": "solves/s", "cells_per_s": 4096 / dt,
            "ms_per_batch_4096": 1e3 * dt, "precision": "bf16 matrix cores, fp32 accumulate",
            "held_out_rel_err": {"p50": float(np.median(err)), "p99": float(np.percentile(err, 99)),
                                 "max": float(err.max()), "cells": int(n_test)},
            "train": {"cells": n_train, "epochs": epochs, "seconds": t_train},
            "labels": {"cells": int(cells.shape[0]), "solves_per_s": cells.shape[0] * sc.N_K / t_label},
            "screening": {"candidates": stats["predicted"], "verified": stats["verified"],
                          "fallback_rate": stats["fallbacks"] / max(1, stats["verified"]),
                          "best_verified_gap_b2_b3": stats["best_gap"],
                          "surrogate_s_per_cell": stats["t_surrogate"] / stats["predicted"],
                          "solve_s_per_cell": stats["t_solve"] / stats["verified"]}}


def variant_precision(mvpb, ctx):
    """4096 Voronoi phases on 128x128, 31x31 plane waves (2N = 1922), 60 k,
    24 bands: FP64, FP32 and BF16 structure factors, and FP32 reduction with
    FP64 Rayleigh-Ritz.  One step per precision after one warm-up."""
    from synth import config3
    cfg = config3()
    cell, M, Q, nb = cfg["cell"], cfg["M"], cfg["Q"], cfg["n_bands"]
    dcell = ctx.cell(cell.phase, cell.props, cell.lattice)
    res, oms = {}, {}
    for name, prec in (("fp64", mvpb.PREC_FP64), ("sf_fp32", mvpb.PREC_SF_FP32), ("sf_bf16", mvpb.PREC_SF_BF16),
                       ("sf_fp32_eig_fp32_rr64", mvpb.PREC_SF_FP32 | mvpb.PREC_EIG_FP32_RR64)):
        out = {}

        def step():
            plan = dcell.plan(M, M, prec)
            out["om"] = plan.solve(Q, nb)
            plan.close()

        dt = run_timed(step, 1, 1, mvpb, "precision " + name)
        res[name] = {"value": Q.shape[0] / dt, "unit": "solves/s", "ms_per_step": 1e3 * dt}
        oms[name] = out["om"]
    return res, oms, cfg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=6, help="k-points timed on the CPU oracle (0 = skip)")
    ap.add_argument("--no-variants", action="store_true", help="only the headline FP64 workload")
    args = ap.parse_args()
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

    def step():
        plan = dcell.plan(M)
        plan.solve_device(Q, nb, om_dev.value)
        plan.close()

    for i in range(args.warmup):
        step()
        progress("fp64 warm-up step", i + 1)
    mvpb.device_synchronize()
    ctx.profile(True)
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

    # roofline of the dominant kernel
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    name, (tot_ms, launches) = dom
    roof = None
    if name == "hetrd_panel" and launches:
        per_item = hetrd_panel_bytes(n)
        bytes_total = Q.shape[0] * sum(per_item) * args.steps
        avg_s = tot_ms / launches / 1e3
        achieved = bytes_total / launches / avg_s / 1e9
        roof = {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_ms": tot_ms / launches, "launches": launches}
    else:
        roof = {"kernel": name, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "avg_launch_ms": tot_ms / max(launches, 1), "launches": launches}

    omega = om_dev.to_numpy(np.float64, (Q.shape[0], nb))
    variants = {}
    om_mixed = om_batch = cfg2 = om_prec = cfg3 = None
    if not args.no_variants:
        variants["mixed_1132_phase"], om_mixed = variant_mixed(mvpb, ctx, dcell, M, Q, nb, args.steps, args.warmup)
        variants["batched_256_cells"], om_batch, cfg2 = variant_batched(mvpb, ctx, max(1, args.steps // 2), 1)
        variants["surrogate_grf_cells"] = variant_surrogate(mvpb, ctx)
        variants["precision_4096_phase"], om_prec, cfg3 = variant_precision(mvpb, ctx)
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Voronoi cell)",
        "config": {"workload": "1132-phase Voronoi cell, 64x64 pixels, 21x21 plane waves (2N=882), "
                               "60 k on G-X-M-G, 18 bands, FP64",
                   "k_points": int(Q.shape[0]), "n_bands": nb, "two_N": n},
        "roofline": roof,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
