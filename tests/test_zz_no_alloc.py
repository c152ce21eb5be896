"""The allocation-free structure-factor entry point against the allocating one.

mvpb_structure_factors_noalloc runs the same kernels as mvpb_structure_factors
with their scratch in a fixed device array; on the same cell, cutoff and
precision the two must agree entry by entry (same kernels, same launch
shapes, same summation order: identical values).  Two calls in a row, the
second at a smaller cutoff on a smaller cell, check that what the first left
in the shared array does not leak into the second.  Each result is also held
to the oracle's subdomain integrals at 1e-13 of the largest entry.
"""
import numpy as np
import pytest

from oracle import mixed_oracle as mo
from synth import Cell, random_iso_props

pytestmark = pytest.mark.gpu


def _rand_cell(nx, ny, P, seed):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, P, (nx, ny)).astype(np.int32)
    return Cell(np.eye(2), phase, random_iso_props(P, rng))


def _oracle_fields(cell, M):
    I = mo.subdomain_integral_tables(cell.phase, cell.n_phases, cell.lattice, M, M)
    J, R, Ph = mo.phase_sum_tables(I, cell.props)
    return np.stack([Ph[0, 0] + Ph[0, 1], Ph[0, 0] - Ph[0, 1], R, J])


def test_noalloc_structure_factors_match_allocating_call():
    from paper_1310_6380_amd import mvpb
    ctx = mvpb.Context(0)
    try:
        cases = [(_rand_cell(48, 40, 6, 11), 9), (_rand_cell(12, 10, 3, 12), 3)]
        for prec in (mvpb.PREC_FP64, mvpb.PREC_SF_PLAIN64):
            for cell, M in cases:
                print("noalloc structure factors", cell.phase.shape, "M", M, "precision", prec, flush=True)
                c = ctx.cell(cell.phase, cell.props, cell.lattice)
                ref = c.structure_factors(M, M, prec)
                n = 4 * (4 * M + 1) ** 2
                buf = mvpb.DeviceBuffer(16 * n)
                c.structure_factors_noalloc(M, M, buf, prec)
                got = buf.to_numpy(np.complex128, ref.shape)
                buf.free()
                assert np.array_equal(got, ref)
                orc = _oracle_fields(cell, M)
                for w in range(4):
                    assert np.max(np.abs(got[w] - orc[w])) <= 1e-13 * np.abs(orc[w]).max(), w
    finally:
        ctx.close()


def test_noalloc_rejects_requests_beyond_the_fixed_scratch():
    from paper_1310_6380_amd import mvpb
    ctx = mvpb.Context(0)
    try:
        cell = _rand_cell(4096, 2, 2, 3)
        c = ctx.cell(cell.phase, cell.props, cell.lattice)
        M = 16   # 64 * 4096 * 65 bytes > 16 MiB
        buf = mvpb.DeviceBuffer(16 * 4 * (4 * M + 1) ** 2)
        with pytest.raises(mvpb.MvpbError) as ei:
            c.structure_factors_noalloc(M, M, buf)
        assert ei.value.code == mvpb.E_NOMEM
        buf.free()
    finally:
        ctx.close()
