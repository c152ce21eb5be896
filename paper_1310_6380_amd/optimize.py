"""Gradient-based band-gap design on top of the mvpb C-ABI.

Design variable: a material fraction x in [0, 1] per pixel of a planar
two-material cell.  The compliance weights and the density of pixel p
interpolate linearly between material A (x = 0) and material B (x = 1).  A
linear combination of two isotropic plane-strain compliances is isotropic
(d22 = d11, d33 = 2 (d11 - d12), no shear-normal coupling), so every pixel
is an isotropic phase of its own, its (E, nu) recovered from the
interpolated d11, d12, and the plans use the isotropic layout.

Objective: the normalised complete gap between bands b and b + 1 (0-based)
over the k list, (min_k w_{b+1} - max_k w_b) / midpoint.  Its gradient comes
from the library's eigenvalue sensitivities (d lambda / d w_f of every
pixel, Sec. 3 eq. (eigenvalueproblem) differentiated), chained through the
interpolation (d lambda / d x_p = sum_f d lambda / d w_f(p) (w_f^B - w_f^A))
and d omega = d lambda / (2 omega).  The smooth objective replaces the max
and min over k by Kreisselmeier-Steinhauser aggregates; the exact one judges
every step (each step is a plain solve on the GPU).  This module only moves
arrays and does the chain rule; the band solves and sensitivities run in the
library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import mvpb


def plane_strain_weights(E, nu):
    """(d11, d12) of isotropic plane strain (d22 = d11, d33 = 2 (d11 - d12))."""
    return (1.0 + nu) * (1.0 - nu) / E, -nu * (1.0 + nu) / E


def iso_from_weights(d11, d12):
    """(E, nu) with the plane-strain compliances d11, d12."""
    r = (d11 + d12) / (d11 - d12)      # = 1 - 2 nu
    nu = 0.5 * (1.0 - r)
    return (1.0 + nu) / (d11 - d12), nu


class Design:
    """Two-material pixel design on a lattice: x [nx, ny] in [0, 1]."""

    def __init__(self, ctx: mvpb.Context, mat_a, mat_b, lattice=None, M: int = 5, Q=None, b: int = 2,
                 n_bands: int = None, ks: float = 200.0):
        self.ctx = ctx
        self.M, self.b = M, b
        self.n_bands = n_bands if n_bands is not None else b + 2
        self.Q = np.asarray(Q if Q is not None else mvpb.kpath_square(20), dtype=np.float64).reshape(-1, 2)
        self.lattice = np.eye(2) if lattice is None else np.asarray(lattice, dtype=np.float64)
        self.ks = ks
        a11, a12 = plane_strain_weights(mat_a[0], mat_a[1])
        b11, b12 = plane_strain_weights(mat_b[0], mat_b[1])
        self.wa = np.array([a11, a12, mat_a[2]])
        self.wb = np.array([b11, b12, mat_b[2]])
        self.solves = 0

    def props(self, x):
        """Per-pixel isotropic rows (E, nu, rho) of the design, pixel (i, j) = phase i ny + j."""
        t = np.asarray(x, dtype=np.float64).reshape(-1, 1)
        w = (1.0 - t) * self.wa[None] + t * self.wb[None]
        E, nu = iso_from_weights(w[:, 0], w[:, 1])
        return np.stack([E, nu, w[:, 2]], axis=1)

    def bands(self, x, vectors=False):
        """Frequencies [n_k, n_bands] (and U) of design x by the plain FP64 solve."""
        nx, ny = np.shape(x)
        phase = np.arange(nx * ny, dtype=np.int32).reshape(nx, ny)
        cell = self.ctx.cell(phase, self.props(x), self.lattice)
        plan = cell.plan(self.M)
        self.solves += self.Q.shape[0]
        out = plan.solve(self.Q, self.n_bands, vectors=vectors)
        if vectors:
            om, U = out
            return om, U, plan, cell
        plan.close()
        cell.close()
        return out

    def gap(self, om):
        """Exact normalised gap between bands b and b+1 over the k list."""
        lo, hi = om[:, self.b].max(), om[:, self.b + 1].min()
        return (hi - lo) / (0.5 * (hi + lo))

    def _ks(self, om):
        """Smooth max_k w_b and min_k w_{b+1} (KS aggregates) and their weights."""
        wb, wc = om[:, self.b], om[:, self.b + 1]
        s = self.ks / wb.max()
        eb = np.exp(s * (wb - wb.max()))
        lo = wb.max() + np.log(eb.sum()) / s
        ec = np.exp(-s * (wc - wc.min()))
        hi = wc.min() - np.log(ec.sum()) / s
        return lo, hi, eb / eb.sum(), ec / ec.sum()

    def smooth_gap(self, om):
        lo, hi, _, _ = self._ks(om)
        return (hi - lo) / (0.5 * (hi + lo))

    def gradient(self, x):
        """(smooth gap, exact gap, d smooth gap / d x [nx, ny]) at design x."""
        om, U, plan, cell = self.bands(x, vectors=True)
        try:
            G = plan.sensitivities(self.Q, om, U, np.shape(x))       # [n_k, n_bands, 7, nx, ny]
        finally:
            plan.close()
            cell.close()
        d = self.wb - self.wa
        # d lambda / d x: fields d11, d12, d13, d22, d23, d33, rho; d22 = d11, d33 = 2 (d11 - d12)
        dlam = (G[:, :, 0] * d[0] + G[:, :, 1] * d[1] + G[:, :, 3] * d[0] + G[:, :, 5] * 2.0 * (d[0] - d[1])
                + G[:, :, 6] * d[2])
        domega = dlam / (2.0 * np.maximum(om, 1e-300))[:, :, None, None]
        lo, hi, pb, pc = self._ks(om)
        dlo = np.tensordot(pb, domega[:, self.b], axes=(0, 0))
        dhi = np.tensordot(pc, domega[:, self.b + 1], axes=(0, 0))
        mid = 0.5 * (hi + lo)
        # g = (hi - lo) / mid
        dg = (dhi - dlo) / mid - (hi - lo) / mid ** 2 * 0.5 * (dhi + dlo)
        return (hi - lo) / mid, self.gap(om), dg

    def optimise(self, x0, iters: int = 10, step: float = 0.25, min_step: float = 1e-3, log=None):
        """Projected gradient ascent with a move limit: x <- clip(x + a g / max|g|);
        a step is kept only if the exact gap of the solved design grows, else the
        move limit is halved.  Returns (x, history of exact gaps)."""
        x = np.clip(np.asarray(x0, dtype=np.float64), 0.0, 1.0)
        _, g_exact, dg = self.gradient(x)
        hist = [g_exact]
        a = step
        for it in range(iters):
            if a < min_step:
                break
            scale = np.abs(dg).max()
            if scale == 0.0:
                break
            trial = np.clip(x + a * dg / scale, 0.0, 1.0)
            gt = self.gap(self.bands(trial))
            if gt > hist[-1]:
                x = trial
                _, g_exact, dg = self.gradient(x)
                hist.append(g_exact)
                a = min(1.0, 1.5 * a)
            else:
                a *= 0.5
            if log:
                log(f"iteration {it + 1}: gap {hist[-1]:.5f}, move limit {a:.4f}")
        return x, hist
