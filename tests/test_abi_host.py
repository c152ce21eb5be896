"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, rejects bad arguments before touching a device, and its k-path helper
matches the seeded generator.  No GPU is used."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1310_6380_amd import mvpb
from synth import kpath_gxmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "mvpb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mvpb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mvpb.load()
    names = _declared_symbols()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mvpb.EXPORTS)
    assert "gfx950" in mvpb.version()


@pytest.mark.parametrize("n_k", [1, 2, 7, 30, 60])
def test_kpath_matches_generator(n_k):
    Q = mvpb.kpath_square(n_k)
    assert np.allclose(Q, kpath_gxmg(n_k), atol=1e-15)


def test_kpath_rejects_bad_arguments():
    lib = mvpb.load()
    assert lib.mvpb_kpath_square(0, None) == mvpb.E_INVALID
    assert "bad" in lib.mvpb_last_error().decode()


def test_null_handles_are_rejected():
    lib = mvpb.load()
    out = ctypes.c_void_p()
    assert lib.mvpb_ctx_create(0, None, 0, None) == mvpb.E_INVALID
    assert lib.mvpb_plan_create(None, 1, 1, 0, ctypes.byref(out)) == mvpb.E_INVALID
    assert lib.mvpb_solve(None, 1, None, 1, None, None, 0) == mvpb.E_INVALID
    assert lib.mvpb_structure_factors(None, 1, 1, 0, None) == mvpb.E_INVALID
    assert lib.mvpb_plan_dofs(None, None, None) == mvpb.E_INVALID
    # destroying NULL handles is a no-op
    assert lib.mvpb_ctx_destroy(None) == 0 and lib.mvpb_cell_destroy(None) == 0
    assert lib.mvpb_plan_destroy(None) == 0


def test_screening_normalizer_round_trip_and_scale():
    """The label standardisation is exactly undone by decode and gives
    unit-variance, zero-mean targets (up to its variance floor)."""
    from paper_1310_6380_amd import screening as sc
    rng = np.random.default_rng(1)
    y = (rng.standard_normal((300, 400)) * rng.uniform(0.01, 3.0, 400) + rng.uniform(0, 5, 400)).astype(np.float32)
    nm = sc.Normalizer(y)
    z = nm.encode(y)
    assert z.dtype == np.float32
    assert np.allclose(z.mean(axis=0), 0.0, atol=1e-4)
    assert np.allclose(z.std(axis=0), y.std(axis=0) / (y.std(axis=0) + 1e-3), rtol=1e-3)
    assert np.allclose(nm.decode(z), y, rtol=1e-5, atol=1e-5)
