"""CPU oracle of the eigenvalue sensitivities of the mixed-variational band
structure (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never does.  It shares no code with the GPU library.

The eigenproblem of Sec. 3, eq. (eigenvalueproblem), in generalized Hermitian
form A U = lambda Omega U with A = H Phi^-1 H* (H* = H^H, H independent of the
material) and U^H Omega U = 1, has for a simple eigenvalue the first-order
change

    d lambda = U^H (dA - lambda dOmega) U,   dA = -H Phi^-1 dPhi Phi^-1 H*,

i.e. d lambda = -S^H dPhi S - lambda U^H dOmega U with the stress modes
S = -Phi^-1 H* U.  The design variables here are the weights of one pixel:
the entries of its engineering-Voigt compliance matrix (the Phi weights of
Sec. 4.1 eq. (ep)) and its density (eq. (eo)).  Changing the weight w_st of
pixel p changes Phi by the pixel's Toeplitz block T_p[r, c] = I_p(n_c - n_r) in
the blocks (s, t) and (t, s); changing rho_p changes Omega by I_2 (x) T_p.  The
matrices below are built densely from those definitions, one pixel at a
time.  Pinned (tests/test_sensitivity_pins.py) against central finite
differences of the band oracle and against Euler's identity for homogeneous
functions.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import mixed_oracle as mo


def field_pairs(ns: int = 3):
    """Voigt pairs (s, t), s <= t, in the order of the weight fields (upper
    triangle row by row); the density is the field after them."""
    return [(s, t) for s in range(ns) for t in range(s, ns)]


def band_sensitivities(phase, weights, rho, lattice, M1, M2, Q, n_bands):
    """d lambda_b / d w_f(pixel) for the planar pixel cell ``phase`` [nx, ny]
    whose phase p has the 3 x 3 Phi weights ``weights[p]`` and density
    ``rho[p]``, at Bloch vector Q.

    Returns (lam [n_bands], G [n_bands, 7, nx, ny]) with the fields f = the six
    pairs of ``field_pairs()`` (w_st = w_ts moves both blocks) and, last, rho.
    Valid for simple eigenvalues.
    """
    phase = np.asarray(phase)
    nx, ny = phase.shape
    weights = np.asarray(weights, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    P = rho.shape[0]
    props = np.stack([np.ones(P), np.zeros(P), rho], axis=1)   # only rho is read from props
    I = mo.subdomain_integral_tables(phase, P, lattice, M1, M2)
    tabs = mo.phase_sum_tables(I, props, phase_weights=weights)
    mats = mo.assemble(I, props, lattice, M1, M2, Q, tables=tabs)
    _, lam, U = mo.solve_k(mats, n_bands, vectors=True)
    S = mo.stress_vector(mats, U)                          # [3N, n_bands]
    N = mats["N"]
    # every pixel's own integral table
    pix = np.arange(nx * ny).reshape(nx, ny)
    Ipix = mo.subdomain_integral_tables(pix, nx * ny, lattice, M1, M2)
    n = mo.plane_wave_indices(M1, M2)
    dm, dq = mo._diff_table(n, M1, M2)
    pairs = field_pairs(3)
    G = np.zeros((n_bands, len(pairs) + 1, nx, ny))
    for i in range(nx):
        for j in range(ny):
            Tp = Ipix[i * ny + j][dm, dq]                      # N x N, row = test, column = trial
            for f, (s, t) in enumerate(pairs):
                dPhi = np.zeros((3 * N, 3 * N), dtype=np.complex128)
                dPhi[s * N:(s + 1) * N, t * N:(t + 1) * N] = Tp
                if s != t:
                    dPhi[t * N:(t + 1) * N, s * N:(s + 1) * N] = Tp
                G[:, f, i, j] = -np.real(np.einsum("rb,rc,cb->b", S.conj(), dPhi, S))
            dOm = np.zeros((2 * N, 2 * N), dtype=np.complex128)
            dOm[:N, :N] = Tp
            dOm[N:, N:] = Tp
            G[:, -1, i, j] = -lam * np.real(np.einsum("rb,rc,cb->b", U.conj(), dOm, U))
    return lam, G


def finite_difference(phase, weights, rho, lattice, M1, M2, Q, n_bands, pixel, field, h=1e-6):
    """Central difference of lambda [n_bands] with respect to field ``field``
    of pixel ``pixel`` = (i, j), that pixel given its own phase; relative
    step h."""
    phase = np.array(phase, copy=True)
    weights = np.asarray(weights, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    i, j = pixel
    p0 = int(phase[i, j])
    P = rho.shape[0]
    phase[i, j] = P                                         # a phase of its own
    pairs = field_pairs(3)
    out = []
    for sign in (1.0, -1.0):
        W = np.concatenate([weights, weights[p0:p0 + 1]], axis=0).copy()
        R = np.concatenate([rho, rho[p0:p0 + 1]]).copy()
        if field < len(pairs):
            s, t = pairs[field]
            step = h * abs(weights[p0, s, s])
            W[P, s, t] += sign * step
            if s != t:
                W[P, t, s] += sign * step
        else:
            step = h * rho[p0]
            R[P] += sign * step
        props = np.stack([np.ones(P + 1), np.zeros(P + 1), R], axis=1)
        I = mo.subdomain_integral_tables(phase, P + 1, lattice, M1, M2)
        tabs = mo.phase_sum_tables(I, props, phase_weights=W)
        mats = mo.assemble(I, props, lattice, M1, M2, Q, tables=tabs)
        A = mo.reduced_operator(mats)
        Om = 0.5 * (mats["Omega"] + mats["Omega"].conj().T)
        out.append(sla.eigh(A, Om, eigvals_only=True, subset_by_index=[0, n_bands - 1]))
    return (out[0] - out[1]) / (2.0 * step)
