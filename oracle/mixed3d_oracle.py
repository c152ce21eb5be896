"""CPU oracle of the three-dimensional mixed-variational band structure
(test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never does.  It shares no code with the GPU library.

Plain, slow, FP64 NumPy/SciPy, every matrix built entry by entry from the
paper's definitions (arXiv:1310.6380) in their three-dimensional form:

* unit cell with lattice vectors h^1, h^2, h^3, x = H_j h^j, Bloch vector
  k = Q_i q^i, q^i . h^j = 2 pi delta_ij: Sec. 2;
* test functions f^{abc} = exp(i (k . x + 2 pi (a H1 + b H2 + c H3))) with
  a, b, c in [-M, M]: Sec. 2.3;
* Galerkin equations for j, k, m, n = 1, 2, 3 with 3 (2M+1)^3 displacement and
  6 (2M+1)^3 stress coefficients: Sec. 2.3, eq. (equationshomogeneous);
* matrix form H S = -lambda Omega U, Phi S = H* U and the eigenproblem
  (H Phi^-1 H*) U = lambda Omega U: Sec. 3, eqs. (equationshomogeneousMatrix),
  (eigenvalueproblem), solved in generalized Hermitian form.

The two-dimensional module (mixed_oracle) writes out eqs. (eh), (eo), (ep) of
Sec. 4.1; the entries here are the same integrals with the third index:
stress unknowns in the order S11, S22, S33, S23, S13, S12, the compliance
weight of the pair (s, t) is c_s c_t D_{jk mn} with c = (1, 1, 1, 2, 2, 2)
(the symmetric pair jk and kj both appear in the sums of the Galerkin
equations), i.e. the engineering-Voigt compliance matrix.

Readings (listed in the design notes): 0-based plane-wave index
I = ((a + M1)(2 M2 + 1) + (b + M2))(2 M3 + 1) + (c + M3); row = test function,
column = trial function; K_n = 2 pi T (Q + n) with T = A^-1; exact voxel
integrals instead of the centroid rule.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .mixed_oracle import _sinc_pi, lame

# stress order of the 6N unknowns and the engineering factors
VOIGT3 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
VOIGT3_FACTOR = [1.0, 1.0, 1.0, 2.0, 2.0, 2.0]


def lattice_quantities3(lattice):
    """A (rows h1, h2, h3), T = A^-1, |Omega| = |det A|, q^i = 2 pi (column i of T)."""
    A = np.asarray(lattice, dtype=np.float64).reshape(3, 3)
    T = np.linalg.inv(A)
    vol = abs(np.linalg.det(A))
    q = 2.0 * np.pi * T.T
    return A, T, vol, q


def plane_wave_indices3(M1, M2, M3):
    out = []
    for a in range(-M1, M1 + 1):
        for b in range(-M2, M2 + 1):
            for c in range(-M3, M3 + 1):
                out.append((a, b, c))
    return np.array(out, dtype=np.int64)


def wavevectors3(T, Q, n):
    """K_n = 2 pi T (Q + n) (rows), so that K_n . x = 2 pi (Q + n) . H."""
    Qn = np.asarray(Q, dtype=np.float64)[None, :] + n.astype(np.float64)
    return 2.0 * np.pi * (Qn @ T.T)


def iso_compliance3(E, nu):
    """Isotropic compliance tensor D_jkmn = 1/(2 mu) [(d_jm d_kn + d_jn d_km)/2
    - lam/(2 mu + 3 lam) d_jk d_mn] (inverse of C = lam d d + mu (d d + d d))."""
    lam, mu = lame(E, nu)
    d = np.eye(3)
    D = np.zeros((3, 3, 3, 3))
    for j in range(3):
        for k in range(3):
            for m in range(3):
                for n in range(3):
                    D[j, k, m, n] = (0.5 * (d[j, m] * d[k, n] + d[j, n] * d[k, m])
                                     - lam / (2.0 * mu + 3.0 * lam) * d[j, k] * d[m, n]) / (2.0 * mu)
    return D


def voigt_weights3(D):
    """6 x 6 weights c_s c_t D_{jk mn} of the Phi blocks (engineering-Voigt compliance)."""
    W = np.zeros((6, 6))
    for s, (j, k) in enumerate(VOIGT3):
        for t, (m, n) in enumerate(VOIGT3):
            W[s, t] = VOIGT3_FACTOR[s] * VOIGT3_FACTOR[t] * D[j, k, m, n]
    return W


def phase_weights3(props):
    """Per-phase 6 x 6 Phi weights from isotropic (E, nu, rho) rows."""
    return np.stack([voigt_weights3(iso_compliance3(E, nu)) for E, nu, _ in props])


def voxel_integrals(phase, n_phases, vol, m_vals, q_vals, r_vals):
    """I_p(m, q, r) = int_{Omega_p} exp(i 2 pi (m H1 + q H2 + r H3)) dx for every
    phase, by direct summation of the exact voxel integral

        |Omega|/(nx ny nz) exp(i 2 pi (m (i+1/2)/nx + q (j+1/2)/ny + r (k+1/2)/nz))
                           sinc(m/nx) sinc(q/ny) sinc(r/nz)

    over the voxels (i, j, k) of each phase.  Returns [n_phases, nm, nq, nr]."""
    phase = np.asarray(phase)
    nx, ny, nz = phase.shape
    m_vals = np.asarray(m_vals, dtype=np.float64)
    q_vals = np.asarray(q_vals, dtype=np.float64)
    r_vals = np.asarray(r_vals, dtype=np.float64)
    ex = np.exp(2j * np.pi * np.outer(m_vals, (np.arange(nx) + 0.5) / nx))
    ey = np.exp(2j * np.pi * np.outer(q_vals, (np.arange(ny) + 0.5) / ny))
    ez = np.exp(2j * np.pi * np.outer(r_vals, (np.arange(nz) + 0.5) / nz))
    fac = (vol / (nx * ny * nz)) * (_sinc_pi(m_vals / nx)[:, None, None] * _sinc_pi(q_vals / ny)[None, :, None]
                                    * _sinc_pi(r_vals / nz)[None, None, :])
    out = np.zeros((n_phases, m_vals.size, q_vals.size, r_vals.size), dtype=np.complex128)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                p = int(phase[i, j, k])
                out[p] += ex[:, i][:, None, None] * ey[:, j][None, :, None] * ez[:, k][None, None, :]
    return out * fac[None]


def integral_tables3(phase, n_phases, lattice, M1, M2, M3):
    """I_p on the (4M1+1) x (4M2+1) x (4M3+1) difference grid."""
    _, _, vol, _ = lattice_quantities3(lattice)
    return voxel_integrals(phase, n_phases, vol, np.arange(-2 * M1, 2 * M1 + 1), np.arange(-2 * M2, 2 * M2 + 1),
                           np.arange(-2 * M3, 2 * M3 + 1))


def _diff3(n, M1, M2, M3):
    """Table indices of n_c - n_r (column = trial, row = test)."""
    d = [n[None, :, a] - n[:, None, a] + 2 * M for a, M in enumerate((M1, M2, M3))]
    return d[0], d[1], d[2]


def assemble3(I_p, props, lattice, M1, M2, M3, Q, weights=None):
    """Dense H (3N x 6N), H* (6N x 3N), Omega (3N x 3N), Phi (6N x 6N) and J
    (N x N) for Bloch vector Q.  ``weights`` overrides the isotropic Phi
    weights with explicit per-phase 6 x 6 matrices."""
    props = np.asarray(props, dtype=np.float64)
    W = phase_weights3(props) if weights is None else np.asarray(weights, dtype=np.float64)
    _, T, _, _ = lattice_quantities3(lattice)
    n = plane_wave_indices3(M1, M2, M3)
    N = n.shape[0]
    K = wavevectors3(T, Q, n)
    d1, d2, d3 = _diff3(n, M1, M2, M3)
    J = I_p.sum(axis=0)[d1, d2, d3]
    R = np.tensordot(props[:, 2], I_p, axes=(0, 0))[d1, d2, d3]
    Pt = np.tensordot(W, I_p, axes=(0, 0))          # [6, 6, nm, nq, nr]
    Phi = np.zeros((6 * N, 6 * N), dtype=np.complex128)
    for s in range(6):
        for t in range(6):
            Phi[s * N:(s + 1) * N, t * N:(t + 1) * N] = Pt[s, t][d1, d2, d3]
    Om = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    for j in range(3):
        Om[j * N:(j + 1) * N, j * N:(j + 1) * N] = R
    # H from <sigma_jk,k, f>: the trial stress S_(ab) enters the u_a equation
    # through d/dx_b and, for a != b, the u_b equation through d/dx_a
    iK = [1j * K[None, :, l] * J for l in range(3)]
    H = np.zeros((3 * N, 6 * N), dtype=np.complex128)
    Hs = np.zeros((6 * N, 3 * N), dtype=np.complex128)
    for s, (a, b) in enumerate(VOIGT3):
        H[a * N:(a + 1) * N, s * N:(s + 1) * N] += iK[b]
        # H* from -<u_(j,k), f> with the engineering factor on the shear rows
        Hs[s * N:(s + 1) * N, a * N:(a + 1) * N] += -iK[b]
        if a != b:
            H[b * N:(b + 1) * N, s * N:(s + 1) * N] += iK[a]
            Hs[s * N:(s + 1) * N, b * N:(b + 1) * N] += -iK[a]
    return dict(H=H, Hs=Hs, Omega=Om, Phi=Phi, J=J, K=K, N=N)


def solve3_k(mats, n_bands, vectors=False):
    """Lowest n_bands of (H Phi^-1 H*) U = lambda Omega U (LAPACK)."""
    cf = sla.cho_factor(mats["Phi"], lower=True)
    A = mats["H"] @ sla.cho_solve(cf, mats["Hs"])
    A = 0.5 * (A + A.conj().T)
    Om = 0.5 * (mats["Omega"] + mats["Omega"].conj().T)
    lam, U = sla.eigh(A, Om, subset_by_index=[0, n_bands - 1])
    om = np.sqrt(np.maximum(lam, 0.0))
    return (om, lam, U) if vectors else (om, lam)


def bands3(phase, props, lattice, M1, M2, M3, Qs, n_bands, I_p=None, weights=None):
    """Band structure of a voxel cell along the Q list (rows Q1, Q2, Q3)."""
    props = np.asarray(props, dtype=np.float64)
    if I_p is None:
        I_p = integral_tables3(phase, props.shape[0], lattice, M1, M2, M3)
    oms, lams = [], []
    for Q in np.asarray(Qs, dtype=np.float64).reshape(-1, 3):
        mats = assemble3(I_p, props, lattice, M1, M2, M3, Q, weights)
        om, lam = solve3_k(mats, n_bands)
        oms.append(om)
        lams.append(lam)
    return np.array(oms), np.array(lams)


def pwe3_bands(phase, props, lattice, M1, M2, M3, Qs, n_bands, I_p=None):
    """Displacement plane-wave (Rayleigh-Ritz) eigenvalues on the same basis:
    int C_jkmn u_m,n conj(v_j,k) = lambda int rho u_j conj(v_j), isotropic
    C_jkmn = lam d_jk d_mn + mu (d_jm d_kn + d_jn d_km)."""
    props = np.asarray(props, dtype=np.float64)
    if I_p is None:
        I_p = integral_tables3(phase, props.shape[0], lattice, M1, M2, M3)
    lam_p, mu_p = lame(props[:, 0], props[:, 1])
    _, T, _, _ = lattice_quantities3(lattice)
    n = plane_wave_indices3(M1, M2, M3)
    N = n.shape[0]
    d1, d2, d3 = _diff3(n, M1, M2, M3)
    Lm = np.tensordot(lam_p, I_p, axes=(0, 0))[d1, d2, d3]
    Mm = np.tensordot(mu_p, I_p, axes=(0, 0))[d1, d2, d3]
    Rm = np.tensordot(props[:, 2], I_p, axes=(0, 0))[d1, d2, d3]
    out = []
    for Q in np.asarray(Qs, dtype=np.float64).reshape(-1, 3):
        K = wavevectors3(T, Q, n)
        Kt, Ka = K[:, None, :], K[None, :, :]
        dot = np.sum(Kt * Ka, axis=2)
        Km = np.zeros((3 * N, 3 * N), dtype=np.complex128)
        Om = np.zeros((3 * N, 3 * N), dtype=np.complex128)
        for j in range(3):
            Om[j * N:(j + 1) * N, j * N:(j + 1) * N] = Rm
            for m in range(3):
                blk = Lm * (Kt[..., j] * Ka[..., m]) + Mm * (Kt[..., m] * Ka[..., j])
                if j == m:
                    blk = blk + Mm * dot
                Km[j * N:(j + 1) * N, m * N:(m + 1) * N] = blk
        Km = 0.5 * (Km + Km.conj().T)
        Om = 0.5 * (Om + Om.conj().T)
        out.append(sla.eigh(Km, Om, eigvals_only=True, subset_by_index=[0, n_bands - 1]))
    return np.array(out)
