"""Eigenfrequency error metric used by the parity tests (test infrastructure).

Relative frequency error per band, except for acoustic modes at or next to
Gamma (frequency below 1e-3 of the top computed band at that k), which are
compared on lambda = omega^2 against an absolute bound scaled by the top band:
|lam - lam_ref| <= 2 tol lam_top.  The function returns the largest error
normalised so that a value <= tol passes.
"""
from __future__ import annotations

import numpy as np


def band_error(omega, omega_ref, floor=1e-3):
    omega = np.asarray(omega, dtype=np.float64)
    ref = np.asarray(omega_ref, dtype=np.float64)
    if omega.shape != ref.shape:
        raise ValueError(f"shape mismatch {omega.shape} vs {ref.shape}")
    ref2 = ref.reshape(-1, ref.shape[-1])
    om2 = omega.reshape(-1, ref.shape[-1])
    top = ref2[:, -1:].copy()
    # a k whose whole reference spectrum is zero (one plane wave at Gamma) is
    # scaled by the largest reference frequency of the set instead
    gmax = float(ref2.max()) if ref2.size else 0.0
    top[top <= 0.0] = gmax if gmax > 0.0 else 1.0
    err = np.zeros_like(ref2)
    big = ref2 >= floor * top
    err[big] = np.abs(om2[big] - ref2[big]) / ref2[big]
    small = ~big
    lam_top = np.broadcast_to(top * top, ref2.shape)
    err[small] = np.abs(om2[small] ** 2 - ref2[small] ** 2) / (2.0 * lam_top[small])
    return float(err.max()) if err.size else 0.0
