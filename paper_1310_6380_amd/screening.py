"""Surrogate-assisted band-gap screening on top of the mvpb C-ABI.

The compute steps run in the library's kernels: labels come from the batched
band solver (batched plan build + one captured launch sequence per size
class), the network is trained and evaluated by the surrogate kernels.  This
module only moves arrays between them and ranks candidates.

Cells are binary 32 x 32 pixel maps (1 = stiff inclusion phase, 0 = matrix)
on the unit square lattice; bands are normalised as omega a / (2 pi c_T) with
c_T the shear speed of the matrix phase, 10 bands at 40 k-points on
Gamma-X-M-Gamma (400 numbers per cell, band-major within each k).
"""
from __future__ import annotations

import time

import numpy as np

from . import mvpb

INCLUSION = (70e9, 0.33, 2700.0)
MATRIX = (3.5e9, 0.35, 1180.0)
N_K = 40
N_BANDS = 10
CUTOFF = 7          # 15 x 15 plane waves


def shear_speed(E, nu, rho):
    return float(np.sqrt(E / (2.0 * (1.0 + nu)) / rho))


C_REF = shear_speed(*MATRIX)


def label_cells(ctx: mvpb.Context, cells: np.ndarray, chunk: int = 512, precision: int = mvpb.PREC_FP64):
    """Normalised bands [n, 400] (float32) of binary cells, by the method."""
    props = np.array([MATRIX, INCLUSION], dtype=np.float64)
    Q = mvpb.kpath_square(N_K)
    out = np.zeros((cells.shape[0], N_K * N_BANDS), dtype=np.float32)
    for c0 in range(0, cells.shape[0], chunk):
        part = cells[c0:c0 + chunk]
        dcells = [ctx.cell(c.astype(np.int32), props) for c in part]
        plans = ctx.plans(dcells, [CUTOFF] * len(dcells), precision)
        om = ctx.solve_batch(plans, [Q] * len(plans), N_BANDS)
        for p in plans:
            p.close()
        for c in dcells:
            c.close()
        out[c0:c0 + len(part)] = (np.stack(om) / (2.0 * np.pi * C_REF)).reshape(len(part), -1)
    return out


class Normalizer:
    """Per-output standardisation of the 400 band targets (the network learns
    (y - mean) / std, whose outputs all have unit scale)."""

    def __init__(self, labels):
        y = np.asarray(labels, dtype=np.float64)
        self.mean = y.mean(axis=0).astype(np.float32)
        self.std = (y.std(axis=0) + 1e-3).astype(np.float32)

    def encode(self, y):
        return ((np.asarray(y, dtype=np.float32) - self.mean) / self.std).astype(np.float32)

    def decode(self, z):
        return (np.asarray(z, dtype=np.float32) * self.std + self.mean).astype(np.float32)


def predict(net: mvpb.Surrogate, cells, norm: Normalizer = None, chunk: int = 4096):
    """Normalised bands [n, 400] predicted by the network."""
    out = np.concatenate([net.infer(cells[i:i + chunk]) for i in range(0, cells.shape[0], chunk)])
    return norm.decode(out) if norm is not None else out


def train(net: mvpb.Surrogate, cells, labels, epochs=20, batch=256, lr=1e-3, seed=0, log=None,
          norm: Normalizer = None, lr_end=None):
    """Adam on shuffled mini-batches; every batch is shifted by a random
    circular translation (the bands of a periodic cell are invariant to it).
    With norm the network is fitted to the standardised targets.  With lr_end
    the step size follows a cosine from lr down to lr_end over the epochs."""
    if norm is not None:
        labels = norm.encode(labels)
    rng = np.random.default_rng(seed)
    n = cells.shape[0]
    losses = []
    for ep in range(epochs):
        lr_ep = lr if lr_end is None else lr_end + 0.5 * (lr - lr_end) * (1.0 + np.cos(np.pi * ep / max(1, epochs)))
        order = rng.permutation(n)
        tot = 0.0
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            idx = order[b0:b0 + batch]
            sy, sx = rng.integers(0, 32, 2)
            x = np.roll(cells[idx], (int(sy), int(sx)), axis=(1, 2))
            tot += net.train_step(x, labels[idx], lr_ep)
            nb += 1
        losses.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep + 1}: loss {losses[-1]:.3e}")
    return losses


def relative_errors(pred, ref, floor=1e-3):
    """Per-cell worst relative band error; modes below floor * (top band at
    that k) are compared against the top band instead (acoustic modes at Gamma)."""
    p = pred.reshape(-1, N_K, N_BANDS).astype(np.float64)
    r = ref.reshape(-1, N_K, N_BANDS).astype(np.float64)
    top = r[:, :, -1:]
    den = np.where(r >= floor * top, r, top)
    return np.max(np.abs(p - r) / den, axis=(1, 2))


def band_gap(bands, b):
    """Normalised complete gap between band b and b+1 (0-based) over the path:
    (min_k w_{b+1} - max_k w_b) / midpoint; negative when the bands overlap."""
    w = bands.reshape(-1, N_K, N_BANDS)
    lo = w[:, :, b].max(axis=1)
    hi = w[:, :, b + 1].min(axis=1)
    return (hi - lo) / (0.5 * (hi + lo))


def mutate(cells, rng, flips=24):
    """Flip a few pixels of each cell, keeping the 0/1 map."""
    out = cells.copy()
    n = out.shape[0]
    iy = rng.integers(0, 32, (n, flips))
    ix = rng.integers(0, 32, (n, flips))
    rows = np.repeat(np.arange(n), flips)
    out[rows, iy.ravel(), ix.ravel()] ^= 1
    return out


def screen(ctx, net, population, b, rounds=3, n_candidates=4096, top_k=16, tol=0.05, seed=0, log=None,
           norm: Normalizer = None):
    """Band-gap maximisation: each round mutates the population into
    n_candidates cells, ranks them by the surrogate's predicted gap, verifies
    the top_k with the plain solve and keeps the best verified cells.  A
    verified cell whose prediction misses the solve by more than tol (relative,
    on the two bands that bound the gap) counts as a fallback: its solved
    bands replace the prediction.  Returns a summary dictionary."""
    rng = np.random.default_rng(seed)
    pop = population.copy()
    best = None
    stats = {"rounds": [], "predicted": 0, "verified": 0, "fallbacks": 0, "t_surrogate": 0.0, "t_solve": 0.0}
    for r in range(rounds):
        parents = pop[rng.integers(0, pop.shape[0], n_candidates)]
        cand = mutate(parents, rng)
        t0 = time.perf_counter()
        pred = predict(net, cand, norm)
        stats["t_surrogate"] += time.perf_counter() - t0
        stats["predicted"] += n_candidates
        gp = band_gap(pred, b)
        top = np.argsort(-gp)[:top_k]
        t0 = time.perf_counter()
        solved = label_cells(ctx, cand[top])
        stats["t_solve"] += time.perf_counter() - t0
        stats["verified"] += top_k
        pw = pred[top].reshape(-1, N_K, N_BANDS)[:, :, b:b + 2]
        sw = solved.reshape(-1, N_K, N_BANDS)[:, :, b:b + 2]
        miss = np.max(np.abs(pw - sw) / np.maximum(sw, 1e-6), axis=(1, 2))
        stats["fallbacks"] += int(np.sum(miss > tol))
        gs = band_gap(solved, b)
        order = np.argsort(-gs)
        pop = cand[top][order[: max(1, min(pop.shape[0], top_k))]]
        if best is None or gs[order[0]] > best[0]:
            best = (float(gs[order[0]]), cand[top][order[0]].copy())
        stats["rounds"].append({"best_verified_gap": float(gs[order[0]]), "best_predicted_gap": float(gp[top[0]]),
                                "median_miss": float(np.median(miss))})
        if log:
            log(f"round {r + 1}: best verified gap {gs[order[0]]:.4f}, predicted {gp[top[0]]:.4f}")
    stats["best_gap"] = best[0]
    stats["best_cell"] = best[1]
    return stats
