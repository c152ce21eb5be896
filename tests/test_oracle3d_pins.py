"""Pins of the three-dimensional CPU oracle, and of the anisotropic weights of
the two-dimensional one, against what mathematics and mechanics fix.

No GPU.  Each test names the part of the oracle it pins and the fact that
fixes it: textbook compliances, brute-force quadrature, the partition of
unity, exact dispersion of homogeneous media (isotropic: c_L |k + G|,
c_T |k + G|; anisotropic: the Christoffel equation), exact dispersion of 1-D
stacks (transfer matrices) along each axis, rigid-body zero modes, the
variational bound against the displacement plane-wave method, and the
symmetry of a cell under a permutation of its axes.
"""
import numpy as np
import pytest

from oracle import mixed3d_oracle as m3
from oracle import mixed_oracle as mo
from oracle import pwe_oracle as pw
from oracle.compare import band_error
from synth import random_iso_props

TRICLINIC = np.array([[1.0, 0.1, -0.05], [0.3, 0.9, 0.1], [-0.2, 0.15, 1.1]])


def _rand_voxels(shape, P, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, P, shape).astype(np.int32), random_iso_props(P, rng)


def test_iso_compliance_is_textbook_engineering_voigt():
    """Isotropic engineering-Voigt compliance: 1/E, -nu/E on the normal block,
    1/mu on the shear diagonal; its inverse is the Lame stiffness matrix."""
    E, nu = 70e9, 0.33
    W = m3.voigt_weights3(m3.iso_compliance3(E, nu))
    lam, mu = mo.lame(E, nu)
    ref = np.zeros((6, 6))
    ref[:3, :3] = -nu / E
    ref[[0, 1, 2], [0, 1, 2]] = 1.0 / E
    ref[[3, 4, 5], [3, 4, 5]] = 1.0 / mu
    assert np.allclose(W, ref, rtol=1e-13, atol=1e-30)
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[[0, 1, 2], [0, 1, 2]] = lam + 2 * mu
    C[[3, 4, 5], [3, 4, 5]] = mu
    assert np.allclose(np.linalg.inv(W), C, rtol=1e-12)


@pytest.mark.parametrize("lattice", [np.eye(3), TRICLINIC])
def test_voxel_integrals_match_quadrature(lattice):
    """Exact voxel integrals = 16-point Gauss-Legendre per voxel in Cartesian
    coordinates x = A^T H (exp is entire), at dG = 2 pi T (m, q, r)."""
    phase, _ = _rand_voxels((3, 2, 2), 2, 4)
    M = 1
    I = m3.integral_tables3(phase, 2, lattice, M, M, M)
    A, T, vol, _ = m3.lattice_quantities3(lattice)
    g, w = np.polynomial.legendre.leggauss(16)
    nx, ny, nz = phase.shape
    ref = np.zeros_like(I)
    grid = np.arange(-2 * M, 2 * M + 1)
    mqr = np.stack(np.meshgrid(grid, grid, grid, indexing="ij"), -1).reshape(-1, 3).astype(float)
    dG = 2 * np.pi * (mqr @ T.T)               # rows: 2 pi T (m, q, r)
    wt = np.einsum("a,b,c->abc", w, w, w).reshape(-1) / 8.0 * vol / (nx * ny * nz)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                H = np.stack(np.meshgrid((i + 0.5 + 0.5 * g) / nx, (j + 0.5 + 0.5 * g) / ny,
                                         (k + 0.5 + 0.5 * g) / nz, indexing="ij"), -1).reshape(-1, 3)
                x = H @ A                      # x = H_j h^j
                ref[phase[i, j, k]] += (wt @ np.exp(1j * (x @ dG.T))).reshape(ref.shape[1:])
    assert np.max(np.abs(I - ref)) < 1e-12 * vol


def test_voxel_partition_of_unity_and_symmetry():
    phase, _ = _rand_voxels((4, 3, 5), 3, 7)
    M = 2
    I = m3.integral_tables3(phase, 3, TRICLINIC, M, M, M)
    vol = abs(np.linalg.det(TRICLINIC))
    S = I.sum(axis=0)
    c = 2 * M
    assert abs(S[c, c, c] - vol) < 1e-14 * vol
    S[c, c, c] = 0.0
    assert np.max(np.abs(S)) < 1e-14 * vol
    assert np.allclose(I[:, ::-1, ::-1, ::-1], np.conj(I), atol=1e-15 * vol)


def test_matrix_structure_and_sizes():
    """3N x 6N H, H* = -H^T, Phi and Omega Hermitian positive definite."""
    phase, props = _rand_voxels((3, 3, 3), 2, 8)
    M = 1
    I = m3.integral_tables3(phase, 2, np.eye(3), M, M, M)
    mats = m3.assemble3(I, props, np.eye(3), M, M, M, [0.1, 0.2, 0.3])
    N = 27
    assert mats["H"].shape == (3 * N, 6 * N) and mats["Phi"].shape == (6 * N, 6 * N)
    assert mats["Omega"].shape == (3 * N, 3 * N)
    assert np.allclose(mats["Hs"], -mats["H"].T)
    for key in ("Phi", "Omega"):
        X = mats[key]
        assert np.allclose(X, X.conj().T, atol=1e-15 * np.abs(X).max())
        assert np.linalg.eigvalsh(X).min() > 0


def _free3(lattice, M, Q, E, nu, rho, nb):
    lam, mu = mo.lame(E, nu)
    cL, cT = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
    _, T, _, q = m3.lattice_quantities3(lattice)
    ks = []
    for n in m3.plane_wave_indices3(M, M, M):
        ks.append(np.linalg.norm((np.asarray(Q) + n) @ q))
    ks = np.array(ks)
    return np.sort(np.concatenate([cL * ks, cT * ks, cT * ks]))[:nb]


@pytest.mark.parametrize("lattice", [np.eye(3), TRICLINIC])
def test_homogeneous_cell_is_folded_free_dispersion(lattice):
    """Homogeneous cell (two phases with equal properties): omega = c_L |k+G|
    and c_T |k+G| (twice) exactly, with q^i the reciprocal vectors."""
    E, nu, rho = 70e9, 0.33, 2700.0
    rng = np.random.default_rng(3)
    phase = rng.integers(0, 2, (4, 4, 4)).astype(np.int32)
    props = np.array([[E, nu, rho], [E, nu, rho]])
    M = 2
    for Q in ([0.25, 0.1, 0.05], [0.5, 0.0, 0.0], [0.31, 0.47, -0.2]):
        om, _ = m3.bands3(phase, props, lattice, M, M, M, np.array([Q]), 16)
        assert band_error(om, _free3(lattice, M, Q, E, nu, rho, 16)[None]) < 1e-12


def test_gamma_three_zero_modes_and_time_reversal():
    phase, props = _rand_voxels((3, 3, 3), 3, 21)
    M = 1
    I = m3.integral_tables3(phase, 3, np.eye(3), M, M, M)
    _, lam = m3.bands3(phase, props, np.eye(3), M, M, M, np.zeros((1, 3)), 5, I_p=I)
    assert np.all(np.abs(lam[0, :3]) < 1e-10 * lam[0, 3])
    Q = np.array([[0.17, 0.33, -0.21]])
    a, _ = m3.bands3(phase, props, np.eye(3), M, M, M, Q, 8, I_p=I)
    b, _ = m3.bands3(phase, props, np.eye(3), M, M, M, -Q, 8, I_p=I)
    assert band_error(a, b) < 1e-12


def _stack(widths, axis, n_tot):
    """Voxel map of a 1-D stack of layers along ``axis`` (one voxel across the others)."""
    ids = np.repeat(np.arange(len(widths)), widths).astype(np.int32)
    shape = [1, 1, 1]
    shape[axis] = n_tot
    return ids.reshape(shape)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_stack_shear_long_wave_speed_exact(axis):
    """1-D bilayer along each axis, one plane wave: the shear bands are
    c = sqrt(<1/mu>^-1 / <rho>) exactly (twice: two polarisations)."""
    props = np.array([(200e9, 0.3, 7800.0), (4e9, 0.38, 1200.0)])
    phase = _stack([6, 10], axis, 16)
    f = np.array([6 / 16, 10 / 16])
    _, mu = mo.lame(props[:, 0], props[:, 1])
    cS = np.sqrt(1.0 / np.sum(f / mu) / np.sum(f * props[:, 2]))
    for Qa in (1e-3, 0.2):
        Q = np.zeros((1, 3))
        Q[0, axis] = Qa
        om, _ = m3.bands3(phase, props, np.eye(3), 0, 0, 0, Q, 2)
        assert np.allclose(om[0], cS * 2 * np.pi * Qa, rtol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_stack_converges_to_transfer_matrix(axis):
    """1-D three-layer stack along each axis: the bands tend to the roots of
    cos(k a) = tr(prod T_i)/2 for P (modulus lam + 2 mu) and S (mu, twice);
    the densest layer is not next to the stiffest, so a transposed Phi or
    Omega table changes the medium."""
    widths = [4, 4, 8]
    props = np.array([(200e9, 0.3, 1500.0), (4e9, 0.38, 7800.0), (60e9, 0.25, 2500.0)])
    phase = _stack(widths, axis, 16)
    layers = [(w / 16, *p) for w, p in zip(widths, props)]
    Qa = 0.3
    Ms = [0, 0, 0]
    Ms[axis] = 40
    Q = np.zeros((1, 3))
    Q[0, axis] = Qa
    om, _ = m3.bands3(phase, props, np.eye(3), *Ms, Q, 6)
    rP = pw.layered_roots(layers, 2 * np.pi * Qa, 4, "P", 4e4, n_scan=8000)
    rS = pw.layered_roots(layers, 2 * np.pi * Qa, 4, "S", 4e4, n_scan=8000)
    ref = np.sort(np.concatenate([rP, rS, rS]))[:6]
    assert np.max(np.abs(om[0] - ref) / ref) < 1.5e-4


def test_mixed_below_pwe_and_pwe_monotone():
    """lam_mixed(M) <= lam_PWE(M) (Loewner bound Phi^-1 <= T[C]) and lam_PWE
    non-increasing in M (Rayleigh-Ritz on nested spaces)."""
    phase, props = _rand_voxels((3, 3, 3), 3, 99)
    Q = np.array([[0.21, 0.08, 0.13], [0.5, 0.37, 0.0]])
    prev = None
    for M in (1, 2):
        I = m3.integral_tables3(phase, 3, np.eye(3), M, M, M)
        _, lm = m3.bands3(phase, props, np.eye(3), M, M, M, Q, 8, I_p=I)
        lp = m3.pwe3_bands(phase, props, np.eye(3), M, M, M, Q, 8, I_p=I)
        assert np.all(lm <= lp * (1 + 1e-12))
        if prev is not None:
            assert np.all(lp <= prev * (1 + 1e-12))
        prev = lp


def test_axis_permutation_invariance():
    """A cubic cell with its axes relabelled (x1, x2, x3) -> (x2, x3, x1) and
    the Bloch vector relabelled alike has the same frequencies."""
    phase, props = _rand_voxels((4, 3, 2), 2, 5)
    perm = np.transpose(phase, (1, 2, 0))       # new axis 0 = old axis 1, ...
    Q = np.array([0.11, 0.27, 0.39])
    a, _ = m3.bands3(phase, props, np.eye(3), 1, 1, 1, Q[None], 8)
    b, _ = m3.bands3(perm, props, np.eye(3), 1, 1, 1, Q[[1, 2, 0]][None], 8)
    assert band_error(a, b) < 1e-12


# ------------------------------------------------------ anisotropic, 2-D

def _christoffel2(W, rho, K):
    """Exact frequencies of a homogeneous in-plane anisotropic medium with
    engineering-Voigt compliance W (S11, S22, S12 order): C = W^-1 as a tensor,
    Gamma_jm = C_jkmn K_k K_n, omega^2 = eig(Gamma) / rho."""
    Cv = np.linalg.inv(W)
    idx = {(0, 0): 0, (1, 1): 1, (0, 1): 2, (1, 0): 2}
    G = np.zeros((2, 2))
    for j in range(2):
        for m in range(2):
            for k in range(2):
                for n in range(2):
                    G[j, m] += Cv[idx[j, k], idx[m, n]] * K[k] * K[n]
    return np.sqrt(np.maximum(np.linalg.eigvalsh(G) / rho, 0.0))


def _aniso_weights(seed):
    """A random symmetric positive-definite engineering-Voigt compliance with
    non-zero normal-shear coupling (S13, S23), scaled like a 10-100 GPa solid."""
    rng = np.random.default_rng(seed)
    B = rng.normal(size=(3, 3))
    return (B @ B.T + 3 * np.eye(3)) * 1e-11


@pytest.mark.parametrize("lattice", [np.eye(2), np.array([[1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])])
def test_anisotropic_homogeneous_cell_is_christoffel(lattice):
    """2-D oracle with explicit per-phase weights (eq. (ep) with D1112, D2212
    non-zero): a homogeneous anisotropic cell gives the Christoffel
    frequencies of every folded plane wave exactly."""
    W = _aniso_weights(1)
    rho = 3000.0
    rng = np.random.default_rng(2)
    phase = rng.integers(0, 2, (6, 6)).astype(np.int32)
    props = np.array([[1e10, 0.3, rho], [1e10, 0.3, rho]])
    M = 2
    I = mo.subdomain_integral_tables(phase, 2, lattice, M, M)
    tabs = mo.phase_sum_tables(I, props, phase_weights=np.stack([W, W]))
    _, T, _, _ = mo.lattice_quantities(lattice)
    n = mo.plane_wave_indices(M, M)
    for Q in ([0.23, 0.11], [0.5, 0.0], [0.0, 0.41]):
        mats = mo.assemble(I, props, lattice, M, M, Q, tables=tabs)
        om, _ = mo.solve_k(mats, 10)
        K = mo.wavevectors(T, Q, n)
        ref = np.sort(np.concatenate([_christoffel2(W, rho, k) for k in K]))[:10]
        assert band_error(om[None], ref[None]) < 1e-12
