"""Many pixel cells in one captured graph (mvpb_solve_cells): plan build and
eigensolve of every (cell, k) pair in one launch, replayed by later calls of
the same shape.  Checked bit for bit against per-cell plans solved through
mvpb_solve_batch, and against the oracle (relative eigenfrequency error
<= 1e-9 in FP64, <= 1e-5 on the mixed path)."""
import numpy as np
import pytest

from oracle import mixed_oracle as mo
from oracle.compare import band_error
from synth import Cell, config2, random_iso_props

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


@pytest.fixture(scope="module")
def ctx():
    from paper_1310_6380_amd import mvpb
    c = mvpb.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _batch(seed, n_incl=6, cutoffs=None):
    """Inclusion cells on 32x32 (several cutoffs) plus random three-phase cells
    on 24x24 and 20x28 sharing cutoffs with them, so that a cutoff group holds
    cells of several grids; k counts differ per cell, one cell has none."""
    cfg = config2(n_cells=n_incl + seed)
    items = cfg["cells"][seed:]
    rng = np.random.default_rng(100 + seed)
    cells = [c["cell"] for c in items]
    Ms = [c["M"] for c in items]
    for nx, ny in ((24, 24), (20, 28)):
        cells.append(Cell(np.eye(2), rng.integers(0, 3, (nx, ny)).astype(np.int32), random_iso_props(3, rng)))
        Ms.append(Ms[0])
    if cutoffs is not None:
        Ms = list(cutoffs)
    Q = cfg["Q"]
    Qs = [Q[i % 3::9][: 3 + (i % 4)] for i in range(len(cells))]
    Qs[1] = Q[:0]
    return cells, Ms, Qs


def _reference(ctx, dcells, Ms, Qs, nb, precision=0):
    plans = ctx.plans(dcells, Ms, precision)
    outs = ctx.solve_batch(plans, Qs, nb)
    for p in plans:
        p.close()
    return outs


def test_solve_cells_matches_batch_and_oracle(ctx):
    nb = 8
    for seed in (0, 3):          # the second call has the same shape: graph replay
        cells, Ms, Qs = _batch(0)
        if seed:
            # same grids, cutoffs and k counts, other materials and maps
            rng = np.random.default_rng(seed)
            cells = [Cell(c.lattice, rng.permutation(c.phase.ravel()).reshape(c.phase.shape).astype(np.int32),
                          random_iso_props(c.props.shape[0], rng)) for c in cells]
        _say("solve_cells call", seed, "cutoffs", Ms, "k counts", [q.shape[0] for q in Qs])
        dcells = [ctx.cell(c.phase, c.props, c.lattice) for c in cells]
        outs = ctx.solve_cells(dcells, Ms, Qs, nb)
        ref = _reference(ctx, dcells, Ms, Qs, nb)
        for o, r in zip(outs, ref):
            assert o.shape == r.shape
            assert np.array_equal(o, r)
        for i in (0, len(cells) - 1):
            c = cells[i]
            orc, _ = mo.bands(c.phase, c.props, c.lattice, Ms[i], Ms[i], Qs[i], nb)
            err = band_error(outs[i], orc)
            _say("  cell", i, "M", Ms[i], "error", err)
            assert err <= TOL64
        for d in dcells:
            d.close()


def test_solve_cells_new_shape_recaptures(ctx):
    """A call of another shape after a captured one: fresh graph, right bands."""
    nb = 6
    for n_incl in (4, 2, 4):
        cells, Ms, Qs = _batch(1, n_incl)
        _say("shape", n_incl, Ms)
        dcells = [ctx.cell(c.phase, c.props, c.lattice) for c in cells]
        outs = ctx.solve_cells(dcells, Ms, Qs, nb)
        ref = _reference(ctx, dcells, Ms, Qs, nb)
        for o, r in zip(outs, ref):
            assert np.array_equal(o, r)
        for d in dcells:
            d.close()


def test_solve_cells_mixed_precision(ctx):
    """Split-BF16 structure factors and the FP32 reduction with FP64
    Rayleigh-Ritz: within 1e-5 of the oracle."""
    from paper_1310_6380_amd import mvpb
    cells, Ms, Qs = _batch(2, 3)
    nb = 8
    prec = mvpb.PREC_SF_BF16X3 | mvpb.PREC_EIG_FP32_RR64
    dcells = [ctx.cell(c.phase, c.props, c.lattice) for c in cells]
    outs = ctx.solve_cells(dcells, Ms, Qs, nb, precision=prec)
    ref = _reference(ctx, dcells, Ms, Qs, nb, prec)
    for i, c in enumerate(cells):
        if Qs[i].shape[0] == 0:
            continue
        assert np.array_equal(outs[i], ref[i])
        orc, _ = mo.bands(c.phase, c.props, c.lattice, Ms[i], Ms[i], Qs[i], nb)
        err = band_error(outs[i], orc)
        _say("  mixed cell", i, "M", Ms[i], "error", err)
        assert err <= 1e-5


def test_solve_cells_under_a_cap_and_rejections(ctx):
    """A workspace cap that splits the eigensolve into several chunks gives the
    same bands; polygon cells, the scalar structure factors and a cap below
    the plan build are refused."""
    from paper_1310_6380_amd import mvpb
    from synth import hex_steel_epoxy
    cells, Ms, Qs = _batch(4, 3, cutoffs=(4, 3, 3, 4, 4))
    nb = 6
    dcells = [ctx.cell(c.phase, c.props, c.lattice) for c in cells]
    full = ctx.solve_cells(dcells, Ms, Qs, nb)
    ran = 0
    for cap in (64 << 20, 32 << 20, 26 << 20, 22 << 20):
        small = mvpb.Context(0, workspace_cap=cap)
        scells = [small.cell(c.phase, c.props, c.lattice) for c in cells]
        try:
            capped = small.solve_cells(scells, Ms, Qs, nb)
            ran += 1
            _say("cap", cap, "ran")
            for o, r in zip(capped, full):
                assert np.array_equal(o, r)
        except mvpb.MvpbError as e:
            _say("cap", cap, "refused")
            assert e.code == mvpb.E_NOMEM
        for c in scells:
            c.close()
        small.close()
    assert ran >= 2
    tiny = mvpb.Context(0, workspace_cap=1 << 20)
    tcells = [tiny.cell(c.phase, c.props, c.lattice) for c in cells]
    with pytest.raises(mvpb.MvpbError) as ei:
        tiny.solve_cells(tcells, Ms, Qs, nb)
    assert ei.value.code == mvpb.E_NOMEM
    with pytest.raises(mvpb.MvpbError) as ei:
        ctx.solve_cells(dcells, Ms, Qs, nb, precision=mvpb.PREC_SF_PLAIN64)
    assert ei.value.code == mvpb.E_UNSUPPORTED
    h = hex_steel_epoxy(16)
    pc = ctx.cell_polygons(h.polygons, h.poly_phase, h.props, h.lattice)
    with pytest.raises(mvpb.MvpbError) as ei:
        ctx.solve_cells([pc], [3], [Qs[0]], nb)
    assert ei.value.code == mvpb.E_UNSUPPORTED
    for c in tcells:
        c.close()
    tiny.close()
