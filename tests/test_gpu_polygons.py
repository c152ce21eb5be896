"""Polygon cells (exact subdomain integrals over polygons, Sec. 4.1 eqs. (eo),
(ep); the hexagonal example of Sec. 5) through the C-ABI against the CPU
oracle.  Bars as for pixel cells: structure factors entry-wise within 1e-12
of the largest entry (edge sums in a different order), eigenfrequencies
within 1e-9 relative (FP64)."""
import json
import os

import numpy as np
import pytest

from oracle import mixed_oracle as mo
from oracle.compare import band_error
from synth import hex_graded_1132, hex_steel_epoxy, kpath_xgjx, random_iso_props

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL64 = 1e-9
OBLIQUE = np.array([[1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])


@pytest.fixture(scope="module")
def ctx():
    from paper_1310_6380_amd import mvpb
    c = mvpb.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _weighted(I, props):
    J, R, Ph = mo.phase_sum_tables(I, props)
    return [Ph[0, 0] + Ph[0, 1], Ph[0, 0] - Ph[0, 1], R, J]


def _pixel_polygons(phase, lattice):
    """Every pixel (i, j) as a parallelogram in Cartesian coordinates
    (x = H1 h1 + H2 h2), counter-clockwise for det A > 0."""
    nx, ny = phase.shape
    h1, h2 = lattice[0], lattice[1]
    polys, ph = [], []
    for i in range(nx):
        for j in range(ny):
            fr = [(i / nx, j / ny), ((i + 1) / nx, j / ny), ((i + 1) / nx, (j + 1) / ny), (i / nx, (j + 1) / ny)]
            polys.append(np.array([a * h1 + b * h2 for a, b in fr]))
            ph.append(int(phase[i, j]))
    return polys, np.array(ph, dtype=np.int32)


def test_polygon_structure_factors_match_oracle(ctx):
    c = hex_steel_epoxy(64)
    M1, M2 = 4, 3
    _say("polygon structure factors", M1, M2)
    F = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice).structure_factors(M1, M2)
    ref = _weighted(mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M1, M2), c.props)
    for w in range(4):
        scale = np.abs(ref[w]).max()
        assert np.max(np.abs(F[w] - ref[w])) <= 1e-12 * scale, w


@pytest.mark.parametrize("lat", ["sq", "ob"])
def test_polygons_of_pixels_equal_pixel_cell(ctx, lat):
    """The same cell given as pixels and as pixel parallelograms: the two
    closed forms (pixel sinc product, polygon edge sum) agree on the GPU."""
    lattice = np.eye(2) if lat == "sq" else OBLIQUE
    rng = np.random.default_rng(7)
    phase = rng.integers(0, 3, (6, 5)).astype(np.int32)
    props = random_iso_props(3, rng)
    polys, ph = _pixel_polygons(phase, lattice)
    _say("pixels as polygons", lat)
    Fp = ctx.cell(phase, props, lattice).structure_factors(3, 3)
    Fg = ctx.cell_polygons(polys, ph, props, lattice).structure_factors(3, 3)
    for w in range(4):
        scale = np.abs(Fp[w]).max()
        assert np.max(np.abs(Fg[w] - Fp[w])) <= 1e-12 * scale, w


def test_hex_polygon_bands_match_oracle(ctx):
    c = hex_steel_epoxy(64)
    M, nb = 5, 12
    Q = kpath_xgjx(13)
    _say("hex polygon bands M =", M)
    om = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice).plan(M).solve(Q, nb)
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    ref, _ = mo.bands(None, c.props, c.lattice, M, M, Q, nb, I_p=I)
    err = band_error(om, ref)
    _say("  band error", err)
    assert err <= TOL64, err


def test_hex_stop_bands_on_gpu_match_paper(ctx):
    """Sec. 5 (golden): the all-angle stop bands of steel cylinders in epoxy."""
    gold = json.load(open(os.path.join(HERE, "golden", "hex_stop_bands.json")))
    c = hex_steel_epoxy(256)
    M = gold["M"]
    _say("hex stop bands on the GPU")
    om = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice).plan(M).solve(kpath_xgjx(61), 12)
    f = om / (2.0 * np.pi) / 1e3
    wide = []
    for b in range(f.shape[1] - 1):
        lo, hi = f[:, b].max(), f[:, b + 1].min()
        if hi - lo >= 10.0:
            wide.append((lo, hi))
    assert len(wide) == len(gold["stop_bands_khz"]), wide
    for (lo, hi), (glo, ghi) in zip(wide, gold["stop_bands_khz"]):
        assert abs(lo - glo) <= 0.02 * glo and abs(hi - ghi) <= 0.02 * ghi, (lo, hi, glo, ghi)


def test_polygon_cell_rejects_bad_input(ctx):
    from paper_1310_6380_amd import mvpb
    c = hex_steel_epoxy(16)
    bad = [
        (c.polygons[:2], c.poly_phase[:2]),                  # cylinder without its hole: does not tile
        ([c.polygons[0][:2]] + c.polygons[1:], c.poly_phase),  # two-vertex polygon
        (c.polygons, np.array([0, 2, 0], dtype=np.int32)),   # phase out of range
    ]
    for polys, ph in bad:
        with pytest.raises(mvpb.MvpbError) as ei:
            ctx.cell_polygons(polys, ph, c.props, c.lattice)
        assert ei.value.code == -1


def test_hex_1132_element_cell_matches_oracle(ctx):
    """The 1132-element hexagonal cell of Sec. 5 (every element its own phase,
    density from the centroid height) at M = 3, where the paper reports
    convergence; 18 bands on X-Gamma-J-X."""
    c = hex_graded_1132()
    M, nb = 3, 18
    Q = kpath_xgjx(9)
    _say("1132-element hexagonal cell, M =", M)
    om = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice).plan(M).solve(Q, nb)
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    ref, _ = mo.bands(None, c.props, c.lattice, M, M, Q, nb, I_p=I)
    err = band_error(om, ref)
    _say("  band error", err)
    assert err <= TOL64, err


def test_polygon_cells_in_batched_solve(ctx):
    """Polygon and pixel cells of different cutoffs through the batched plan
    build and the batched solve: the same frequencies as one solve each."""
    c = hex_steel_epoxy(32)
    pc = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice)
    rng = np.random.default_rng(3)
    phase = rng.integers(0, 2, (8, 8)).astype(np.int32)
    xc = ctx.cell(phase, random_iso_props(2, rng), np.eye(2))
    cells, Ms = [pc, xc, pc], [3, 4, 5]
    Qs = [kpath_xgjx(5), np.array([[0.1, 0.2], [0.5, 0.0]]), kpath_xgjx(4)]
    _say("polygon cells in a batched solve")
    plans = ctx.plans(cells, Ms)
    outs = ctx.solve_batch(plans, Qs, 8)
    for cell, M, Q, om in zip(cells, Ms, Qs, outs):
        ref = cell.plan(M).solve(Q, 8)
        assert np.max(np.abs(om - ref) / np.maximum(np.abs(ref), 1e-300 + np.abs(ref).max() * 1e-12)) <= 1e-9


def test_hex_all_242_eigenvalues(ctx):
    """Sec. 5 computes every eigenvalue of the steel/epoxy cell at M = 5
    (2N = 242): all 242 bands per k beyond the Rayleigh-Ritz block (the
    frequencies and vectors straight from the FP64 tridiagonal eigenpairs),
    against the oracle, the vectors Omega-orthonormal."""
    c = hex_steel_epoxy(64)
    M, nb = 5, 242
    Q = kpath_xgjx(7)
    _say("hex all eigenvalues, M =", M)
    plan = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice).plan(M)
    om, U = plan.solve(Q, nb, vectors=True)
    assert om.shape == (7, 242) and np.all(np.isfinite(om))
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    ref, _ = mo.bands(None, c.props, c.lattice, M, M, Q, nb, I_p=I)
    err = band_error(om, ref)
    _say("  band error", err)
    assert err <= TOL64, err
    tabs = mo.phase_sum_tables(I, c.props)
    mats = mo.assemble(I, c.props, c.lattice, M, M, Q[3], tables=tabs)
    G = U[3].conj() @ mats["Omega"] @ U[3].T
    assert np.max(np.abs(G - np.eye(nb))) <= 1e-8
    # the largest band count with the Rayleigh-Ritz step and the smallest without agree on their bands
    o64 = plan.solve(Q, 64)
    o65 = plan.solve(Q, 65)
    assert band_error(o65[:, :64], o64) <= TOL64
