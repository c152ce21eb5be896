"""CPU oracle for the mixed-variational phononic band structure (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never does.  It shares no code with the GPU library.

Plain, slow, FP64 NumPy/SciPy.  Every matrix is built entry by entry from its
definition in the paper (Srivastava, "Fast phononic band-structure
calculations through a GPU accelerated mixed-variational formulation",
arXiv:1310.6380):

* lattice, reciprocal basis and Bloch vector: Sec. 2 (first display equation,
  k = Q_i q^i) and Sec. 4 (the matrix [A]_jk = h^j . e^k, T = A^-1);
* Bloch-Fourier basis: Sec. 2.3 (test functions f^{alpha beta gamma}) and
  Sec. 4, eq. (approximation2d);
* Galerkin system: Sec. 2.3, eq. (equationshomogeneous) and Sec. 3,
  eq. (equationshomogeneousMatrix);
* matrix entries: Sec. 4.1, eqs. (eh), (eo), (ep);
* isotropic plane-strain compliance: Sec. 4, the D_jkmn display;
* eigenproblem: Sec. 3, eq. (eigenvalueproblem), solved here in its
  generalized Hermitian form A U = lambda Omega U, A = H Phi^-1 H*.

Readings where the paper is ambiguous or garbled (listed in the design notes):
* H is 2N x 3N (rows: displacement test functions, columns: stress
  coefficients); the size printed in Sec. 4.1 is its transpose.
* Row = test function (theta, eta), column = trial function (alpha, beta); the
  integrand f is exp(i (K^{ab} - K^{te}) . x).
* K_n = 2 pi T (Q + n), i.e. the T(0,1) = T_12 form of the Sec. 5 listing.
* 0-based plane-wave index I = (alpha + M1)(2 M2 + 1) + (beta + M2).
* Subdomain integrals are exact closed forms over pixels or polygons rather
  than the centroid rule of Sec. 3 (the rule is an approximation of the same
  integrals).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

# --------------------------------------------------------------------------
# Lattice and basis  (Sec. 2; Sec. 4 eq. approximation2d)
# --------------------------------------------------------------------------


def lattice_quantities(lattice):
    """A_jk = h^j . e^k (rows of ``lattice`` are h1, h2), T = A^-1, |Omega| = |det A|,
    reciprocal vectors q^i with q^i . h^j = 2 pi delta_ij (q^i = 2 pi * column i of T)."""
    A = np.asarray(lattice, dtype=np.float64)
    T = np.linalg.inv(A)
    area = abs(np.linalg.det(A))
    q = 2.0 * np.pi * T.T          # row i = q^i
    return A, T, area, q


def plane_wave_indices(M1, M2):
    """All n = (alpha, beta), alpha in [-M1, M1], beta in [-M2, M2], alpha-major order.

    Index I = (alpha + M1)(2 M2 + 1) + (beta + M2)  (0-based form of Sec. 4.1's I_1).
    """
    out = []
    for a in range(-M1, M1 + 1):
        for b in range(-M2, M2 + 1):
            out.append((a, b))
    return np.array(out, dtype=np.int64)


def wavevectors(T, Q, n):
    """K_n = 2 pi T (Q + n) for each plane wave n (rows), Q fractional (Q1, Q2).

    With x = A^T H this gives K_n . x = 2 pi (Q + n) . H, the phase of the
    Bloch-Fourier test function of Sec. 2.3 in 2-D.
    """
    Qn = np.asarray(Q, dtype=np.float64)[None, :] + n.astype(np.float64)
    return 2.0 * np.pi * (Qn @ T.T)


# --------------------------------------------------------------------------
# Compliance  (Sec. 4, isotropic plane strain)
# --------------------------------------------------------------------------


def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def plane_strain_compliance(E, nu):
    """Full 2x2x2x2 tensor D_jkmn = 1/(2 mu) [ (d_jm d_kn + d_jn d_km)/2 - lam/(2(mu+lam)) d_jk d_mn ]."""
    lam, mu = lame(E, nu)
    d = np.eye(2)
    D = np.zeros((2, 2, 2, 2))
    for j in range(2):
        for k in range(2):
            for m in range(2):
                for n in range(2):
                    D[j, k, m, n] = (0.5 * (d[j, m] * d[k, n] + d[j, n] * d[k, m])
                                     - lam / (2.0 * (mu + lam)) * d[j, k] * d[m, n]) / (2.0 * mu)
    return D


# stress components in the order of S = {S11, S22, S12} (Sec. 4.1)
_VOIGT = [(0, 0), (1, 1), (0, 1)]
_VOIGT_FACTOR = [1.0, 1.0, 2.0]


def phi_weights(D):
    """3x3 matrix of the compliance factors multiplying the integrals in eq. (ep):
    entry (s, t) = c_s c_t D_{jk mn} with (jk) = stress s, (mn) = stress t and
    c = (1, 1, 2), e.g. (1,1) -> D1111, (1,3) -> 2 D1112, (3,3) -> 4 D1212."""
    W = np.zeros((3, 3))
    for s, (j, k) in enumerate(_VOIGT):
        for t, (m, n) in enumerate(_VOIGT):
            W[s, t] = _VOIGT_FACTOR[s] * _VOIGT_FACTOR[t] * D[j, k, m, n]
    return W


def phase_phi_weights(props):
    """Per-phase 3x3 weight matrices from (E, nu, rho) rows."""
    return np.stack([phi_weights(plane_strain_compliance(E, nu)) for E, nu, _ in props])


# --------------------------------------------------------------------------
# Subdomain integrals  I_p(dG) = int_{Omega_p} exp(i dG . x) dx   (Sec. 3, Sec. 4.1)
# --------------------------------------------------------------------------


def _sinc_pi(t):
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    nz = t != 0.0
    out[nz] = np.sin(np.pi * t[nz]) / (np.pi * t[nz])
    return out


def pixel_integrals(phase, n_phases, area, m_vals, q_vals):
    """I_p(m, q) for every phase p and every fractional frequency (m, q).

    dG = 2 pi T (m, q), so dG . x = 2 pi (m H1 + q H2).  Pixel (i, j) covers
    H1 in [i/nx, (i+1)/nx], H2 in [j/ny, (j+1)/ny]; its exact integral is

        |Omega|/(nx ny) * exp(i 2 pi (m (i+1/2)/nx + q (j+1/2)/ny))
                        * sinc(m/nx) * sinc(q/ny),      sinc(t) = sin(pi t)/(pi t).

    The sum over the pixels of each phase is done by direct summation.
    Returns complex array [n_phases, len(m_vals), len(q_vals)].
    """
    phase = np.asarray(phase)
    nx, ny = phase.shape
    m_vals = np.asarray(m_vals, dtype=np.float64)
    q_vals = np.asarray(q_vals, dtype=np.float64)
    ci = (np.arange(nx) + 0.5) / nx
    cj = (np.arange(ny) + 0.5) / ny
    ex = np.exp(2j * np.pi * np.outer(m_vals, ci))       # [nm, nx]
    ey = np.exp(2j * np.pi * np.outer(q_vals, cj))       # [nq, ny]
    shape_fac = np.outer(_sinc_pi(m_vals / nx), _sinc_pi(q_vals / ny)) * (area / (nx * ny))
    out = np.zeros((n_phases, m_vals.size, q_vals.size), dtype=np.complex128)
    for i in range(nx):
        for j in range(ny):
            p = int(phase[i, j])
            out[p] += np.outer(ex[:, i], ey[:, j])
    out *= shape_fac[None]
    return out


def polygon_integral(verts, dG):
    """int over a simple polygon (vertices CCW, Cartesian) of exp(i dG . x) dA;
    for clockwise vertices the same sum is minus that integral (a hole).

    Divergence theorem with F = -i dG/|dG|^2 exp(i dG.x):  for dG != 0,
        sum over edges e of (-i/|dG|^2) (dG . n_e) L_e exp(i dG . m_e) sinc_u(dG . t_e L_e / 2),
    with m_e the edge midpoint, L_e its length, t_e the unit tangent, n_e the
    outward unit normal and sinc_u(u) = sin(u)/u; for dG = 0 the area.
    ``dG`` is [..., 2]; returns complex array of shape dG.shape[:-1].
    """
    V = np.asarray(verts, dtype=np.float64)
    dG = np.asarray(dG, dtype=np.float64)
    shp = dG.shape[:-1]
    g = dG.reshape(-1, 2)
    out = np.zeros(g.shape[0], dtype=np.complex128)
    area = 0.5 * np.sum(V[:, 0] * np.roll(V[:, 1], -1) - np.roll(V[:, 0], -1) * V[:, 1])
    g2 = np.sum(g * g, axis=1)
    zero = g2 == 0.0
    for e in range(V.shape[0]):
        a = V[e]
        b = V[(e + 1) % V.shape[0]]
        L = np.hypot(*(b - a))
        if L == 0.0:
            continue
        t = (b - a) / L
        nrm = np.array([t[1], -t[0]])            # outward for CCW order
        mid = 0.5 * (a + b)
        u = (g @ t) * (0.5 * L)
        sinc = np.ones_like(u)
        nz = u != 0.0
        sinc[nz] = np.sin(u[nz]) / u[nz]
        term = (g @ nrm) * L * np.exp(1j * (g @ mid)) * sinc
        out[~zero] += (-1j / g2[~zero]) * term[~zero]
    out[zero] = area
    return out.reshape(shp)


# --------------------------------------------------------------------------
# Assembly  (Sec. 4.1, eqs. eh, eo, ep; Sec. 3 eq. equationshomogeneousMatrix)
# --------------------------------------------------------------------------


def _diff_table(n, M1, M2):
    """For row (test) index r and column (trial) index c: the frequency n_c - n_r
    shifted to non-negative table indices."""
    dm = n[None, :, 0] - n[:, None, 0] + 2 * M1
    dq = n[None, :, 1] - n[:, None, 1] + 2 * M2
    return dm, dq


def subdomain_integral_tables(cell_phase, n_phases, lattice, M1, M2):
    """I_p on the full (4 M1 + 1) x (4 M2 + 1) difference grid, pixel cells."""
    _, _, area, _ = lattice_quantities(lattice)
    m_vals = np.arange(-2 * M1, 2 * M1 + 1)
    q_vals = np.arange(-2 * M2, 2 * M2 + 1)
    return pixel_integrals(cell_phase, n_phases, area, m_vals, q_vals)


def polygon_integral_tables(polygons, poly_phase, n_phases, lattice, M1, M2):
    """I_p on the full (4 M1 + 1) x (4 M2 + 1) difference grid for a polygon
    cell: the sum over the polygons of phase p of their integrals (clockwise
    polygons subtract), at dG = 2 pi T (m, q) (Sec. 4: K_n = 2 pi T (Q + n))."""
    _, T, _, _ = lattice_quantities(lattice)
    m_vals = np.arange(-2 * M1, 2 * M1 + 1)
    q_vals = np.arange(-2 * M2, 2 * M2 + 1)
    mq = np.stack(np.meshgrid(m_vals, q_vals, indexing="ij"), axis=-1).astype(np.float64)
    dG = 2.0 * np.pi * (mq @ T.T)
    out = np.zeros((n_phases, m_vals.size, q_vals.size), dtype=np.complex128)
    for verts, p in zip(polygons, poly_phase):
        out[int(p)] += polygon_integral(verts, dG)
    return out


def phase_sum_tables(I_p, props, phase_weights=None):
    """Phase sums on the difference grid: int_Omega w(x) f = sum_p w_p I_p for
    w = 1 (J), rho (R) and the nine Phi weights of eq. (ep)."""
    props = np.asarray(props, dtype=np.float64)
    W = phase_weights if phase_weights is not None else phase_phi_weights(props)
    J = I_p.sum(axis=0)
    R = np.tensordot(props[:, 2], I_p, axes=(0, 0))
    Ph = np.tensordot(W, I_p, axes=(0, 0))      # [3, 3, nm, nq]
    return J, R, Ph


def assemble(I_p, props, lattice, M1, M2, Q, phase_weights=None, tables=None):
    """Dense H (2N x 3N), H* (3N x 2N), Omega (2N x 2N), Phi (3N x 3N) and the
    plain overlap J (N x N) = int_Omega f, for the Bloch vector Q.

    Rows index test functions (theta, eta), columns trial functions (alpha, beta);
    every entry uses f = exp(i (K^{ab} - K^{te}) . x) integrated over the cell,
    i.e. the difference-grid table at n_ab - n_te.  ``phase_weights`` overrides
    the isotropic Phi weights with explicit per-phase 3x3 matrices.
    """
    _, T, _, _ = lattice_quantities(lattice)
    n = plane_wave_indices(M1, M2)
    N = n.shape[0]
    K = wavevectors(T, Q, n)                     # [N, 2]
    Jt, Rt, Pht = tables if tables is not None else phase_sum_tables(I_p, props, phase_weights)
    dm, dq = _diff_table(n, M1, M2)
    J = Jt[dm, dq]                               # int_Omega f
    R = Rt[dm, dq]                               # int_Omega rho f

    # Phi: eq. (ep); block (s, t) = int c_s c_t D_{s t} f
    Phi = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    for s in range(3):
        for t in range(3):
            Phi[s * N:(s + 1) * N, t * N:(t + 1) * N] = Pht[s, t][dm, dq]

    # Omega: eq. (eo); block-diagonal in the two displacement components
    Om = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    Om[:N, :N] = R
    Om[N:, N:] = R

    # H: eq. (eh), from <sigma_jk,k, f^{te}>:  d/dx_k of the trial function
    # brings i K^{ab}_k (column index)
    iK1 = 1j * K[None, :, 0] * J
    iK2 = 1j * K[None, :, 1] * J
    H = np.zeros((2 * N, 3 * N), dtype=np.complex128)
    H[:N, 0:N] = iK1            # u1-row, S11
    H[:N, 2 * N:3 * N] = iK2    # u1-row, S12
    H[N:, N:2 * N] = iK2        # u2-row, S22
    H[N:, 2 * N:3 * N] = iK1    # u2-row, S12

    # H*: from -<u_(j,k), f^{te}> with the engineering factor 2 on the 12 row
    Hs = np.zeros((3 * N, 2 * N), dtype=np.complex128)
    Hs[0:N, :N] = -iK1
    Hs[N:2 * N, N:] = -iK2
    Hs[2 * N:, :N] = -iK2
    Hs[2 * N:, N:] = -iK1
    return dict(H=H, Hs=Hs, Omega=Om, Phi=Phi, J=J, K=K, N=N)


# --------------------------------------------------------------------------
# Eigenproblem  (Sec. 3 eq. eigenvalueproblem)
# --------------------------------------------------------------------------


def reduced_operator(mats):
    """A = H Phi^-1 H*, by a Cholesky solve with Phi; made exactly Hermitian."""
    cf = sla.cho_factor(mats["Phi"], lower=True)
    X = sla.cho_solve(cf, mats["Hs"])
    A = mats["H"] @ X
    return 0.5 * (A + A.conj().T)


def solve_k(mats, n_bands, vectors=False):
    """Lowest n_bands of A U = lambda Omega U (LAPACK generalized Hermitian solver).

    Returns (omega, lam[, U]) with omega = sqrt(max(lam, 0)) ascending and
    U^H Omega U = I.
    """
    A = reduced_operator(mats)
    Om = mats["Omega"]
    Om = 0.5 * (Om + Om.conj().T)
    lam, U = sla.eigh(A, Om, subset_by_index=[0, n_bands - 1])
    om = np.sqrt(np.maximum(lam, 0.0))
    if vectors:
        return om, lam, U
    return om, lam


def stress_vector(mats, U):
    """S = -Phi^-1 H* U (Sec. 3, after eq. eigenvalueproblem)."""
    return -sla.cho_solve(sla.cho_factor(mats["Phi"], lower=True), mats["Hs"] @ U)


def bands(cell_phase, props, lattice, M1, M2, Qs, n_bands, I_p=None, vectors=False):
    """Band structure of a pixel cell along the Q list: omega [n_k, n_bands]."""
    props = np.asarray(props, dtype=np.float64)
    if I_p is None:
        I_p = subdomain_integral_tables(cell_phase, props.shape[0], lattice, M1, M2)
    tables = phase_sum_tables(I_p, props)
    oms, lams, Us = [], [], []
    for Q in np.asarray(Qs, dtype=np.float64).reshape(-1, 2):
        mats = assemble(I_p, props, lattice, M1, M2, Q, tables=tables)
        r = solve_k(mats, n_bands, vectors=vectors)
        oms.append(r[0])
        lams.append(r[1])
        if vectors:
            Us.append(r[2])
    if vectors:
        return np.array(oms), np.array(lams), Us
    return np.array(oms), np.array(lams)
