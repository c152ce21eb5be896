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
    t0 = time.perf_counter()
    ref, _ = mo.bands(cell.phase, cell.props, cell.lattice, M, M, Q[idx], nb)
    dt = time.perf_counter() - t0
    err = band_error(omega_gpu[idx], ref)
    return {
        "value": n_sample / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": f"{n_sample} of the {Q.shape[0]} k-points of the same cell (incl. its subdomain integrals), "
                  f"NumPy/SciPy LAPACK, {dt:.1f} s",
    }, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=6, help="k-points timed on the CPU oracle (0 = skip)")
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

    for _ in range(args.warmup):
        step()
    mvpb.device_synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
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
    if args.cpu_sample > 0:
        cb, err = cpu_baseline(cell, M, Q, nb, omega, args.cpu_sample)
        out["cpu_baseline"] = cb
        out["max_rel_freq_err_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
