"""Displacement plane-wave expansion (PWE) and 1-D transfer-matrix dispersion.

TEST INFRASTRUCTURE ONLY (see mixed_oracle).  These are independent methods
used to pin the mixed-variational oracle:

* the PWE is the displacement-only Rayleigh-Ritz method on the same
  Bloch-Fourier basis; its eigenvalues bound the exact ones from above and
  bound the mixed-variational ones from above at the same cutoff;
* the transfer-matrix relation is the exact dispersion relation of a 1-D
  layered medium (for two layers this is Rytov's relation).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.optimize import brentq

from .mixed_oracle import (_diff_table, lame, lattice_quantities, plane_wave_indices,
                           subdomain_integral_tables, wavevectors)


def pwe_bands(phase, props, lattice, M1, M2, Qs, n_bands):
    """Lowest eigenvalues of K U = lambda Omega U with the plane-strain stiffness
    C_jkmn = lam d_jk d_mn + mu (d_jm d_kn + d_jn d_km) and the weak form
    int sigma_jk conj(v_j,k) = lambda int rho u_j conj(v_j)."""
    props = np.asarray(props, dtype=np.float64)
    I_p = subdomain_integral_tables(phase, props.shape[0], lattice, M1, M2)
    lam_p, mu_p = lame(props[:, 0], props[:, 1])
    Lt = np.tensordot(lam_p, I_p, axes=(0, 0))
    Mt = np.tensordot(mu_p, I_p, axes=(0, 0))
    Rt = np.tensordot(props[:, 2], I_p, axes=(0, 0))
    _, T, _, _ = lattice_quantities(lattice)
    n = plane_wave_indices(M1, M2)
    N = n.shape[0]
    dm, dq = _diff_table(n, M1, M2)
    Lm, Mm, Rm = Lt[dm, dq], Mt[dm, dq], Rt[dm, dq]
    out = []
    for Q in np.asarray(Qs, dtype=np.float64).reshape(-1, 2):
        K = wavevectors(T, Q, n)
        Kt = K[:, None, :]        # test  (row)
        Ka = K[None, :, :]        # trial (column)
        dot = np.sum(Kt * Ka, axis=2)
        Kmat = np.zeros((2 * N, 2 * N), dtype=np.complex128)
        for j in range(2):
            for m in range(2):
                blk = Lm * (Kt[..., j] * Ka[..., m]) + Mm * (Kt[..., m] * Ka[..., j])
                if j == m:
                    blk = blk + Mm * dot
                Kmat[j * N:(j + 1) * N, m * N:(m + 1) * N] = blk
        Om = np.zeros((2 * N, 2 * N), dtype=np.complex128)
        Om[:N, :N] = Rm
        Om[N:, N:] = Rm
        Kmat = 0.5 * (Kmat + Kmat.conj().T)
        Om = 0.5 * (Om + Om.conj().T)
        lam = sla.eigh(Kmat, Om, eigvals_only=True, subset_by_index=[0, n_bands - 1])
        out.append(lam)
    return np.array(out)


def layered_trace(omega, layers, wave):
    """Half-trace of the unit-cell transfer matrix of a 1-D stack.

    ``layers``: list of (thickness, E, nu, rho); ``wave`` 'P' uses the
    plane-strain modulus lam + 2 mu, 'S' uses mu.  Each layer maps
    (u, sigma) by [[cos(kd), sin(kd)/(Z w)], [-Z w sin(kd), cos(kd)]],
    kd = w d / c, Z = rho c.
    """
    Mtot = np.eye(2)
    for d, E, nu, rho in layers:
        lam, mu = lame(E, nu)
        mod = lam + 2.0 * mu if wave == "P" else mu
        c = np.sqrt(mod / rho)
        Z = rho * c
        th = omega * d / c
        Lm = np.array([[np.cos(th), np.sin(th) / (Z * omega)],
                       [-Z * omega * np.sin(th), np.cos(th)]])
        Mtot = Lm @ Mtot
    return 0.5 * np.trace(Mtot)


def layered_roots(layers, kx, n_roots, wave, w_max, n_scan=200000):
    """Lowest n_roots of cos(kx a) = half-trace(w) for 0 < w < w_max, found by a
    dense scan and bisection refinement (simple roots only)."""
    a = sum(L[0] for L in layers)
    target = np.cos(kx * a)
    ws = np.linspace(w_max / n_scan, w_max, n_scan)
    f = np.array([layered_trace(w, layers, wave) for w in ws]) - target
    roots = []
    for i in range(len(ws) - 1):
        if f[i] == 0.0:
            roots.append(ws[i])
        elif f[i] * f[i + 1] < 0.0:
            roots.append(brentq(lambda w: layered_trace(w, layers, wave) - target, ws[i], ws[i + 1],
                                xtol=1e-14 * ws[i + 1], rtol=1e-15))
        if len(roots) >= n_roots:
            break
    return np.array(roots)
