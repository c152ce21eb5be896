"""Stress modes S = -Phi^-1 H* U (Sec. 3, after eq. (eigenvalueproblem)) through
the C-ABI: against the oracle's dense Cholesky solve with Phi on the GPU's own
U (so degenerate bands need no special care), and against the Galerkin
relation H S = -lambda Omega U that the pair (U, S) satisfies.  Bar: 1e-10 of
the largest entry (explicit inverse factors against a Cholesky solve)."""
import numpy as np
import pytest

from oracle import mixed_oracle as mo
from synth import hex_steel_epoxy, random_iso_props

pytestmark = pytest.mark.gpu

OBLIQUE = np.array([[1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])


@pytest.fixture(scope="module")
def ctx():
    from paper_1310_6380_amd import mvpb
    c = mvpb.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _check(plan, I, props, lattice, M, Q, nb):
    om, U = plan.solve(Q, nb, vectors=True)
    S = plan.stress(Q, U)
    for t, q in enumerate(Q):
        mats = mo.assemble(I, props, lattice, M, M, q)
        V = U[t].T                                   # [2N, nb]
        ref = mo.stress_vector(mats, V)              # [3N, nb]
        err = np.max(np.abs(S[t].T - ref)) / np.max(np.abs(ref))
        _say("  k", t, "stress error", err)
        assert err <= 1e-10, err
        lam = om[t] ** 2
        rel = np.linalg.norm(mats["H"] @ S[t].T + mats["Omega"] @ V * lam[None]) / \
            np.linalg.norm(mats["Omega"] @ V * lam[None])
        assert rel <= 1e-9, rel


@pytest.mark.parametrize("lat", ["sq", "ob"])
def test_stress_modes_pixel_cell(ctx, lat):
    lattice = np.eye(2) if lat == "sq" else OBLIQUE
    rng = np.random.default_rng(21)
    phase = rng.integers(0, 3, (8, 8)).astype(np.int32)
    props = random_iso_props(3, rng)
    M, nb = 3, 8
    Q = np.array([[0.21, 0.35], [0.5, 0.5], [0.03, -0.11]])
    _say("stress modes, pixel cell", lat)
    plan = ctx.cell(phase, props, lattice).plan(M)
    I = mo.subdomain_integral_tables(phase, 3, lattice, M, M)
    _check(plan, I, props, lattice, M, Q, nb)


def test_stress_modes_hex_polygon_cell(ctx):
    c = hex_steel_epoxy(64)
    M, nb = 4, 10
    Q = np.array([[0.3, 0.1], [2.0 / 3.0, 1.0 / 3.0]])
    _say("stress modes, hexagonal polygon cell")
    plan = ctx.cell_polygons(c.polygons, c.poly_phase, c.props, c.lattice).plan(M)
    I = mo.polygon_integral_tables(c.polygons, c.poly_phase, c.n_phases, c.lattice, M, M)
    _check(plan, I, c.props, c.lattice, M, Q, nb)
