"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

No GPU.  Each test names the part of the oracle it pins and the fact that
fixes it (closed forms, exact dispersion relations, variational bounds,
symmetries, brute-force quadrature).
"""
import json
import os

import numpy as np
import pytest
import scipy.special as sps

from oracle import mixed_oracle as mo
from oracle import pwe_oracle as pw
from oracle.compare import band_error
from synth import Cell, circle_cell, layered_cell, random_iso_props, rng_for

HERE = os.path.dirname(os.path.abspath(__file__))
OBLIQUE = np.array([[1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])   # hexagonal lattice, a = 1


def _reciprocal_by_cross_product(lattice):
    """q^1, q^2 from the cross-product formula of Sec. 2 with h^3 = e3."""
    h1 = np.array([lattice[0, 0], lattice[0, 1], 0.0])
    h2 = np.array([lattice[1, 0], lattice[1, 1], 0.0])
    h3 = np.array([0.0, 0.0, 1.0])
    q1 = 2 * np.pi * np.cross(h2, h3) / np.dot(h1, np.cross(h2, h3))
    q2 = 2 * np.pi * np.cross(h3, h1) / np.dot(h2, np.cross(h3, h1))
    return q1[:2], q2[:2]


def _cross2(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]


def _random_cell(nx, ny, n_phases, seed):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, n_phases, (nx, ny)).astype(np.int32)
    return phase, random_iso_props(n_phases, rng)


# ---------------------------------------------------------------- lattice

def test_reciprocal_basis_matches_cross_product():
    """O2: q^i . h^j = 2 pi delta_ij, q^i equal to the Sec. 2 cross-product formula."""
    for lat in (np.eye(2), OBLIQUE, np.array([[1.3, 0.2], [-0.4, 0.9]])):
        _, T, area, q = mo.lattice_quantities(lat)
        q1, q2 = _reciprocal_by_cross_product(lat)
        assert np.allclose(q[0], q1, atol=1e-14) and np.allclose(q[1], q2, atol=1e-14)
        assert np.allclose(q @ lat.T, 2 * np.pi * np.eye(2), atol=1e-13)
        assert np.isclose(area, abs(_cross2(lat[0], lat[1])))


def test_wavevector_is_bloch_plus_reciprocal():
    """K_n = k + alpha q^1 + beta q^2 with k = Q_i q^i (Sec. 2)."""
    lat = np.array([[1.3, 0.2], [-0.4, 0.9]])
    _, T, _, _ = mo.lattice_quantities(lat)
    q1, q2 = _reciprocal_by_cross_product(lat)
    n = mo.plane_wave_indices(2, 1)
    Q = np.array([0.21, -0.37])
    K = mo.wavevectors(T, Q, n)
    ref = (Q[0] + n[:, :1]) * q1[None] + (Q[1] + n[:, 1:]) * q2[None]
    assert np.allclose(K, ref, atol=1e-13)


# ---------------------------------------------------------------- compliance

def test_plane_strain_compliance_identities():
    """P11 + O4: textbook plane-strain compliances and the isotropic identities."""
    for E, nu in [(70e9, 0.33), (3.5e9, 0.35), (200e9, 0.2)]:
        lam, mu = mo.lame(E, nu)
        W = mo.phi_weights(mo.plane_strain_compliance(E, nu))
        d11, d12, d33 = W[0, 0], W[0, 1], W[2, 2]
        assert np.isclose(d11, (1 + nu) * (1 - nu) / E, rtol=1e-14)
        assert np.isclose(d12, -nu * (1 + nu) / E, rtol=1e-14)
        assert np.isclose(d33, 1 / mu, rtol=1e-14)
        assert np.isclose(d33, 2 * (d11 - d12), rtol=1e-14)
        assert np.isclose(d11 + d12, 1 / (2 * (lam + mu)), rtol=1e-14)
        assert W[0, 2] == 0 and W[1, 2] == 0 and np.allclose(W, W.T)
        # inverse of the plane-strain stiffness in engineering Voigt form
        C = np.array([[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]])
        assert np.allclose(W @ C, np.eye(3), atol=1e-14)


# ---------------------------------------------------------------- subdomain integrals

def _gauss_legendre_tables(phase, n_phases, lattice, M1, M2, order=16):
    """Brute-force I_p(m, q) by Gauss-Legendre on each pixel, in Cartesian x."""
    nx, ny = phase.shape
    q1, q2 = _reciprocal_by_cross_product(lattice)
    jac = abs(_cross2(lattice[0], lattice[1]))
    g, w = np.polynomial.legendre.leggauss(order)
    u = 0.5 * (g + 1.0)
    w = 0.5 * w
    out = np.zeros((n_phases, 4 * M1 + 1, 4 * M2 + 1), dtype=complex)
    for i in range(nx):
        for j in range(ny):
            H1 = (i + u) / nx
            H2 = (j + u) / ny
            HH1, HH2 = np.meshgrid(H1, H2, indexing="ij")
            WW = np.outer(w, w) * jac / (nx * ny)
            X = HH1[..., None] * lattice[0] + HH2[..., None] * lattice[1]
            for a, m in enumerate(range(-2 * M1, 2 * M1 + 1)):
                for b, q in enumerate(range(-2 * M2, 2 * M2 + 1)):
                    dG = m * q1 + q * q2
                    out[phase[i, j], a, b] += np.sum(WW * np.exp(1j * (X @ dG)))
    return out


@pytest.mark.parametrize("lattice", [np.eye(2), OBLIQUE])
def test_pixel_integrals_match_quadrature(lattice):
    """P4: exact pixel closed form == 16-point Gauss-Legendre (integrand entire)."""
    phase, props = _random_cell(5, 4, 3, 7)
    M1, M2 = 2, 1
    I = mo.subdomain_integral_tables(phase, 3, lattice, M1, M2)
    ref = _gauss_legendre_tables(phase, 3, lattice, M1, M2)
    assert np.max(np.abs(I - ref)) < 1e-13 * abs(_cross2(lattice[0], lattice[1]))


def test_pixel_integrals_partition_and_symmetry():
    """P3 + P4: sum_p I_p(dG) = |Omega| delta_{dG,0};  I(-dG) = conj I(dG)."""
    phase, _ = _random_cell(12, 9, 4, 3)
    M1, M2 = 5, 4
    I = mo.subdomain_integral_tables(phase, 4, OBLIQUE, M1, M2)
    area = abs(np.linalg.det(OBLIQUE))
    S = I.sum(axis=0)
    ref = np.zeros_like(S)
    ref[2 * M1, 2 * M2] = area
    assert np.max(np.abs(S - ref)) < 1e-15 * 100
    assert np.allclose(I[:, ::-1, ::-1], I.conj(), atol=1e-16 * 100)
    # zero frequency = phase areas
    counts = np.bincount(phase.ravel(), minlength=4)
    assert np.allclose(I[:, 2 * M1, 2 * M2].real, area * counts / phase.size, atol=1e-15)


def test_polygon_union_of_pixels_equals_pixels():
    """P4: a phase given as pixel squares (as polygons) matches the pixel closed form."""
    phase, _ = _random_cell(4, 4, 2, 11)
    M = 3
    I = mo.subdomain_integral_tables(phase, 2, np.eye(2), M, M)
    g = np.arange(-2 * M, 2 * M + 1)
    dG = 2 * np.pi * np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1)
    acc = np.zeros((2, g.size, g.size), dtype=complex)
    for i in range(4):
        for j in range(4):
            x0, y0 = i / 4, j / 4
            sq = [(x0, y0), (x0 + .25, y0), (x0 + .25, y0 + .25), (x0, y0 + .25)]
            acc[phase[i, j]] += mo.polygon_integral(sq, dG)
    assert np.max(np.abs(acc - I)) < 1e-14


def test_polygon_disk_limit_is_bessel():
    """P4: regular n-gon of circumradius R -> 2 pi R J1(|q| R)/|q| as n grows."""
    R = 0.3
    qs = np.array([[0.0, 0.0], [3.0, 1.0], [-7.0, 4.0], [12.0, -2.0]])
    nv = 4096
    t = 2 * np.pi * np.arange(nv) / nv
    verts = np.stack([0.5 + R * np.cos(t), 0.5 + R * np.sin(t)], axis=1)
    val = mo.polygon_integral(verts, qs) * np.exp(-1j * (qs @ np.array([0.5, 0.5])))
    qn = np.linalg.norm(qs, axis=1)
    ref = np.where(qn > 0, 2 * np.pi * R * sps.j1(qn * R) / np.where(qn > 0, qn, 1), np.pi * R * R)
    # polygon area deficit of a 4096-gon is ~ (2 pi / n)^2 / 6 relative
    assert np.max(np.abs(val - ref)) < 1e-6


def test_polygon_triangle_matches_quadrature():
    """P4: polygon formula on a triangle vs a Dunavant-free brute-force sum."""
    tri = np.array([[0.1, 0.2], [0.8, 0.3], [0.3, 0.9]])
    qs = np.array([[2.0, -1.0], [5.0, 3.0], [0.0, 4.0]])
    val = mo.polygon_integral(tri, qs)
    # map the unit square to the triangle (Duffy) and integrate with Gauss-Legendre
    g, w = np.polynomial.legendre.leggauss(40)
    u = 0.5 * (g + 1)
    w = 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    WW = np.outer(w, w)
    a, b, c = tri
    P = a + U[..., None] * (b - a) + (U * V)[..., None] * (c - b)
    jac = abs(_cross2(b - a, c - b)) * U
    ref = np.array([np.sum(WW * jac * np.exp(1j * (P @ q))) for q in qs])
    assert np.max(np.abs(val - ref)) < 1e-12


# ---------------------------------------------------------------- assembled matrices

def test_matrix_structure_and_sizes():
    """Sec. 4.1 sizes (golden), P5: Phi, Omega Hermitian PD; H* = -H^T; J = |Omega| I;
    Phi and Omega independent of Q."""
    gold = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    assert 2 * mo.plane_wave_indices(5, 5).shape[0] == gold["eigenvalues_at_M5"]
    phase, props = _random_cell(8, 8, 3, 5)
    M = 2
    I = mo.subdomain_integral_tables(phase, 3, OBLIQUE, M, M)
    m1 = mo.assemble(I, props, OBLIQUE, M, M, np.array([0.13, 0.31]))
    m2 = mo.assemble(I, props, OBLIQUE, M, M, np.array([-0.4, 0.05]))
    N = (2 * M + 1) ** 2
    assert m1["H"].shape == (2 * N, 3 * N) and m1["Hs"].shape == (3 * N, 2 * N)
    assert m1["Phi"].shape == (3 * N, 3 * N) and m1["Omega"].shape == (2 * N, 2 * N)
    area = abs(np.linalg.det(OBLIQUE))
    assert np.allclose(m1["J"], area * np.eye(N), atol=1e-15)
    for key in ("Phi", "Omega"):
        X = m1[key]
        assert np.allclose(X, X.conj().T, atol=1e-15 * np.abs(X).max())
        assert np.linalg.eigvalsh(0.5 * (X + X.conj().T)).min() > 0
        assert np.array_equal(m1[key], m2[key])
    assert np.allclose(m1["Hs"], -m1["H"].T, atol=1e-14 * np.abs(m1["H"]).max())


# ---------------------------------------------------------------- eigenproblem

def _free_dispersion(lattice, M1, M2, Q, E, nu, rho, nb):
    lam, mu = mo.lame(E, nu)
    cL, cT = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
    q1, q2 = _reciprocal_by_cross_product(lattice)
    ks = []
    for a in range(-M1, M1 + 1):
        for b in range(-M2, M2 + 1):
            ks.append(np.linalg.norm((Q[0] + a) * q1 + (Q[1] + b) * q2))
    ks = np.array(ks)
    return np.sort(np.concatenate([cL * ks, cT * ks]))[:nb]


@pytest.mark.parametrize("lattice", [np.eye(2), OBLIQUE])
def test_homogeneous_cell_is_folded_free_dispersion(lattice):
    """P1 (and P2: two phases with equal properties): omega = c_{L,T} |k + G| exactly."""
    E, nu, rho = 70e9, 0.33, 2700.0
    cell = circle_cell(10, 0.3, inc=(E, nu, rho), mat=(E, nu, rho))
    M = 3
    for Q in ([0.25, 0.1], [0.5, 0.0], [0.0, 0.0], [0.31, 0.47]):
        om, _ = mo.bands(cell.phase, cell.props, lattice, M, M, np.array([Q]), 14)
        ref = _free_dispersion(lattice, M, M, Q, E, nu, rho, 14)
        assert band_error(om, ref[None]) < 1e-12


def test_gamma_zero_modes_and_time_reversal():
    """P6: exactly two zero eigenvalues at Gamma (rigid translations); omega(-k) = omega(k)."""
    phase, props = _random_cell(8, 8, 3, 21)
    M = 3
    I = mo.subdomain_integral_tables(phase, 3, np.eye(2), M, M)
    om, lam = mo.bands(phase, props, np.eye(2), M, M, np.array([[0.0, 0.0]]), 4, I_p=I)
    assert abs(lam[0, 0]) < 1e-10 * lam[0, 2] and abs(lam[0, 1]) < 1e-10 * lam[0, 2]
    assert lam[0, 2] > 1e-3 * lam[0, 3]
    Q = np.array([[0.17, 0.33]])
    a, _ = mo.bands(phase, props, np.eye(2), M, M, Q, 8, I_p=I)
    b, _ = mo.bands(phase, props, np.eye(2), M, M, -Q, 8, I_p=I)
    assert band_error(a, b) < 1e-12


def test_bilayer_shear_long_wave_speed_exact():
    """P7: 1-D bilayer, M = 0: the shear band is c = sqrt(<1/mu>^-1 / <rho>) exactly."""
    props = [(200e9, 0.3, 7800.0), (4e9, 0.38, 1200.0)]
    cell = layered_cell([6, 10], props, 16)
    f = np.array([6 / 16, 10 / 16])
    _, mu = mo.lame(np.array([p[0] for p in props]), np.array([p[1] for p in props]))
    rho = np.array([p[2] for p in props])
    cS = np.sqrt(1.0 / np.sum(f / mu) / np.sum(f * rho))
    for Q1 in (1e-3, 0.2):
        om, _ = mo.bands(cell.phase, cell.props, cell.lattice, 0, 0, np.array([[Q1, 0.0]]), 1)
        assert np.isclose(om[0, 0], cS * 2 * np.pi * Q1, rtol=1e-13)


@pytest.mark.parametrize("widths,props", [
    ([6, 10], [(200e9, 0.3, 7800.0), (4e9, 0.38, 1200.0)]),
    # three layers with the densest layer not adjacent to the stiffest one: a
    # transposed Phi or Omega table changes this medium
    ([4, 4, 8], [(200e9, 0.3, 1500.0), (4e9, 0.38, 7800.0), (60e9, 0.25, 2500.0)]),
])
def test_layered_converges_to_transfer_matrix(widths, props):
    """P7: 1-D stacks -> roots of cos(k a) = tr(prod T_i)/2 (Rytov for two layers)."""
    cell = layered_cell(widths, props, sum(widths))
    layers = [(w / sum(widths), *p) for w, p in zip(widths, props)]
    Q1 = 0.3
    kx = 2 * np.pi * Q1
    om, _ = mo.bands(cell.phase, cell.props, cell.lattice, 40, 0, np.array([[Q1, 0.0]]), 5)
    rP = pw.layered_roots(layers, kx, 4, "P", 4e4, n_scan=8000)
    rS = pw.layered_roots(layers, kx, 4, "S", 4e4, n_scan=8000)
    ref = np.sort(np.concatenate([rP, rS]))[:4]
    # M = 40 leaves ~6e-5 truncation error on the P band of the three-layer stack;
    # a transposed Phi or Omega table moves these bands by more than 5 %
    assert np.max(np.abs(om[0, :4] - ref) / ref) < 1.5e-4


def test_mixed_below_pwe_and_pwe_monotone():
    """P8: lam_mixed(M) <= lam_PWE(M) (Loewner bound) and lam_PWE non-increasing in M
    (Rayleigh-Ritz on nested spaces); on a cell without symmetry."""
    phase, props = _random_cell(6, 6, 3, 99)
    Q = np.array([[0.21, 0.08], [0.5, 0.37]])
    nb = 8
    prev = None
    for M in (1, 2, 3, 4):
        _, lm = mo.bands(phase, props, np.eye(2), M, M, Q, nb)
        lp = pw.pwe_bands(phase, props, np.eye(2), M, M, Q, nb)
        assert np.all(lm <= lp * (1 + 1e-12))
        if prev is not None:
            assert np.all(lp <= prev * (1 + 1e-12))
        prev = lp


def test_mixed_eigenvalues_rise_with_cutoff():
    """P9 (observed, unproven): lam_mixed non-decreasing in M on this cell."""
    phase, props = _random_cell(6, 6, 3, 99)
    Q = np.array([[0.21, 0.08]])
    prev = None
    for M in (1, 2, 3, 4, 5):
        _, lm = mo.bands(phase, props, np.eye(2), M, M, Q, 8)
        if prev is not None:
            assert np.all(lm >= prev * (1 - 1e-12))
        prev = lm


def test_circular_shift_and_c4v_symmetry():
    """P10: shifting the pixel map leaves omega unchanged; the circle cell has
    omega(Q1, Q2) = omega(Q2, Q1)."""
    phase, props = _random_cell(8, 8, 3, 4)
    Q = np.array([[0.2, 0.1], [0.45, 0.3]])
    a, _ = mo.bands(phase, props, np.eye(2), 3, 3, Q, 8)
    b, _ = mo.bands(np.roll(phase, (3, -2), axis=(0, 1)), props, np.eye(2), 3, 3, Q, 8)
    assert band_error(a, b) < 1e-12
    cell = circle_cell(16, 0.3)
    a, _ = mo.bands(cell.phase, cell.props, cell.lattice, 3, 3, Q, 8)
    b, _ = mo.bands(cell.phase, cell.props, cell.lattice, 3, 3, Q[:, ::-1], 8)
    assert band_error(a, b) < 1e-12


def test_eigenvectors_residual_and_normalisation():
    """P12: ||A U - Omega U Lam|| <= 1e-12 ||A||; U^H Omega U = I; same spectrum as
    numpy's standard solver on L^-1 A L^-H."""
    phase, props = _random_cell(8, 8, 3, 8)
    M = 3
    I = mo.subdomain_integral_tables(phase, 3, np.eye(2), M, M)
    mats = mo.assemble(I, props, np.eye(2), M, M, np.array([0.3, 0.2]))
    om, lam, U = mo.solve_k(mats, 10, vectors=True)
    A = mo.reduced_operator(mats)
    Om = mats["Omega"]
    assert np.linalg.norm(A @ U - Om @ U * lam[None]) <= 1e-12 * np.linalg.norm(A)
    assert np.allclose(U.conj().T @ Om @ U, np.eye(10), atol=1e-12)
    L = np.linalg.cholesky(Om)
    Li = np.linalg.inv(L)
    ev = np.linalg.eigvalsh(Li @ A @ Li.conj().T)[:10]
    assert np.allclose(ev, lam, rtol=1e-10, atol=1e-12 * np.abs(ev).max())
    # stress eigenvector satisfies the second Galerkin equation Phi S + H* U = 0
    S = mo.stress_vector(mats, U)
    assert np.linalg.norm(mats["Phi"] @ S + mats["Hs"] @ U) < 1e-12 * np.linalg.norm(mats["Hs"] @ U)


def _stop_bands_khz(omega):
    """Complete gaps between consecutive bands over the sampled path, in kHz."""
    f = np.asarray(omega) / (2.0 * np.pi) / 1e3
    out = []
    for b in range(f.shape[1] - 1):
        lo, hi = f[:, b].max(), f[:, b + 1].min()
        if hi > lo:
            out.append((b, lo, hi))
    return out


def _wide_gaps(gaps, min_width_khz=10.0):
    return [(lo, hi) for _, lo, hi in gaps if hi - lo >= min_width_khz]


def test_hex_steel_epoxy_stop_bands_match_paper():
    """P14 (Sec. 5, golden): steel cylinders in epoxy on the hexagonal lattice,
    M = 5, X-Gamma-J-X: the all-angle stop bands the paper states."""
    from synth import hex_steel_epoxy, kpath_xgjx, iso_from_c11_c44
    gold = json.load(open(os.path.join(HERE, "golden", "hex_stop_bands.json")))
    c = hex_steel_epoxy(256)
    assert np.allclose(c.lattice[0], [gold["a_m"], 0.0])
    assert np.allclose(c.props[1], iso_from_c11_c44(*gold["steel_c11_c44_rho"]))
    assert np.allclose(c.props[0], iso_from_c11_c44(*gold["epoxy_c11_c44_rho"]))
    M = gold["M"]
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    om, _ = mo.bands(None, c.props, c.lattice, M, M, kpath_xgjx(31), 12, I_p=I)
    wide = _wide_gaps(_stop_bands_khz(om))
    assert len(wide) == len(gold["stop_bands_khz"]), wide
    for (lo, hi), (glo, ghi) in zip(wide, gold["stop_bands_khz"]):
        assert abs(lo - glo) <= 0.02 * glo and abs(hi - ghi) <= 0.02 * ghi, (lo, hi, glo, ghi)


def test_polygon_cell_partition_and_holes():
    """P3 for polygon cells: a cylinder cut out of the cell as a clockwise
    polygon leaves sum_p I_p = |Omega| delta (signed areas tile the cell), and
    I(-dG) = conj I(dG)."""
    from synth import hex_steel_epoxy
    c = hex_steel_epoxy(64)
    M = 4
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    _, _, area, _ = mo.lattice_quantities(c.lattice)
    J = I.sum(axis=0)
    ref = np.zeros_like(J)
    ref[2 * M, 2 * M] = area
    assert np.max(np.abs(J - ref)) <= 1e-14 * area
    assert np.allclose(I[:, ::-1, ::-1], I.conj(), atol=1e-15 * area)
    # phase areas: the n-gon has the disk's area
    assert abs(I[1, 2 * M, 2 * M].real - np.pi * (2e-3) ** 2) <= 1e-12 * area


def test_hex_1132_element_cell_tiles_the_cell():
    """The 1132-element hexagonal cell (Sec. 5): exactly 1132 elements, every
    one its own phase, counter-clockwise, tiling the primitive cell (partition
    of unity of the oracle's polygon integrals), density 10^6 x centroid x2."""
    from synth import hex_graded_1132
    c = hex_graded_1132()
    assert len(c.polygons) == 1132 and c.n_phases == 1132
    areas = np.array([0.5 * np.sum(v[:, 0] * np.roll(v[:, 1], -1) - np.roll(v[:, 0], -1) * v[:, 1])
                      for v in c.polygons])
    assert np.all(areas > 0)
    _, _, area, _ = mo.lattice_quantities(c.lattice)
    assert abs(areas.sum() - area) <= 1e-12 * area
    cent_y = np.array([np.mean(v[:, 1]) for v in c.polygons])
    assert np.allclose(c.props[:, 2], 1e6 * cent_y)
    M = 2
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    J = I.sum(axis=0)
    ref = np.zeros_like(J)
    ref[2 * M, 2 * M] = area
    assert np.max(np.abs(J - ref)) <= 1e-13 * area
