"""Gradient-based band-gap design (eigenvalue sensitivities of the HIP path
chained through a two-material pixel interpolation).

* the analytic gradient of the smooth gap matches central differences of the
  smooth gap computed by plain GPU solves along a random direction;
* projected gradient ascent raises the exact complete gap of a seeded
  Gaussian-random-field start, every accepted step verified by a solve, and
  the final gap is confirmed by the CPU oracle.
"""
import numpy as np
import pytest

from oracle import mixed_oracle as mo
from synth import INCLUSION_PROPS, MATRIX_PROPS, grf_phase_map, kpath_gxmg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1310_6380_amd import mvpb
    c = mvpb.Context(0)
    yield c
    c.close()


def _design(ctx, M=4, nk=16, b=2):
    from paper_1310_6380_amd.optimize import Design
    return Design(ctx, MATRIX_PROPS, INCLUSION_PROPS, M=M, Q=kpath_gxmg(nk), b=b)


def test_gradient_matches_finite_differences(ctx):
    rng = np.random.default_rng(41)
    x = rng.uniform(0.2, 0.8, (12, 12))
    v = rng.normal(size=x.shape)
    v /= np.abs(v).max()
    d = _design(ctx)
    sg, _, dg = d.gradient(x)
    h = 1e-4
    fp = d.smooth_gap(d.bands(x + h * v))
    fm = d.smooth_gap(d.bands(x - h * v))
    fd = (fp - fm) / (2 * h)
    an = float(np.sum(dg * v))
    print("directional derivative", an, "finite difference", fd, flush=True)
    assert abs(an - fd) <= 1e-4 * abs(fd)


def test_gradient_ascent_opens_the_gap(ctx):
    rng = np.random.default_rng(42)
    x0 = grf_phase_map(16, 3.0, 0.45, rng).astype(np.float64)
    d = _design(ctx, M=4, nk=16, b=2)
    x, hist = d.optimise(x0, iters=10, log=lambda s: print(s, flush=True))
    print("gap history", hist, "solves", d.solves, flush=True)
    assert all(b > a for a, b in zip(hist, hist[1:]))
    assert hist[-1] > hist[0] + 0.02
    # the final design's bands (every pixel its own isotropic phase) by the oracle
    phase = np.arange(x.size, dtype=np.int32).reshape(x.shape)
    ref, _ = mo.bands(phase, d.props(x), np.eye(2), d.M, d.M, d.Q, d.n_bands)
    assert abs(d.gap(ref) - hist[-1]) <= 1e-8
