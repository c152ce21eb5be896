"""Pins of the parity metric (oracle/compare.py) and of the PWE helper.

No GPU.  Every parity assertion of the GPU tests goes through band_error, so
its value is fixed here by hand-computed cases, one per branch: the relative
frequency error, the eigenvalue comparison for modes far below the top band
at their k (the acoustic modes at or next to Gamma), the all-zero spectrum,
and the shape check.  A metric that returned 0, divided by the computed value
instead of the reference, took the top band from the computed values, or
dropped the eigenvalue branch would fail one of these.
"""
import numpy as np
import pytest

from oracle import mixed_oracle as mo
from oracle import pwe_oracle as pw
from oracle.compare import band_error
from synth import circle_cell


def test_relative_branch_exact_values():
    ref = np.array([[1.0, 2.0, 4.0]])
    assert band_error(ref, ref) == 0.0
    # 10 % off on the first band: relative to the reference, not to the computed value
    assert band_error(np.array([[1.1, 2.0, 4.0]]), ref) == pytest.approx(0.1, rel=1e-14)
    assert band_error(np.array([[2.0, 2.0, 4.0]]), ref) == pytest.approx(1.0, rel=1e-14)
    # the largest error over every band and k is returned, not a mean
    om = np.array([[1.0, 2.2, 4.0], [1.0, 2.0, 4.04]])
    assert band_error(om, np.vstack([ref, ref])) == pytest.approx(0.1, rel=1e-13)
    # sign does not matter
    assert band_error(np.array([[0.9, 2.0, 4.0]]), ref) == pytest.approx(0.1, rel=1e-13)


def test_eigenvalue_branch_for_modes_far_below_the_top_band():
    # top band 10, floor 1e-3 * 10 = 1e-2: the 1e-5 mode is compared on lambda
    # against 2 * lam_top = 200
    ref = np.array([[1e-5, 1.0, 10.0]])
    om = np.array([[0.5, 1.0, 10.0]])
    assert band_error(om, ref) == pytest.approx((0.25 - 1e-10) / 200.0, rel=1e-12)
    # a mode at the floor itself is compared relatively
    ref2 = np.array([[1e-2, 1.0, 10.0]])
    assert band_error(np.array([[1.1e-2, 1.0, 10.0]]), ref2) == pytest.approx(0.1, rel=1e-12)
    # the floor follows the top band of each k (from the reference), not the
    # largest frequency of the set: at k 0 the floor is 2e-3, so 3e-3 is
    # compared relatively (error 1); with the set's maximum (2000) it would be
    # compared on lambda and pass
    refk = np.array([[3e-3, 0.5, 2.0], [1.0, 1.5, 2000.0]])
    omk = np.array([[6e-3, 0.5, 2.0], [1.0, 1.5, 2000.0]])
    assert band_error(omk, refk) == pytest.approx(1.0, rel=1e-12)
    # both k on the lambda branch: the larger of the two normalised errors
    refl = np.array([[1e-3, 0.5, 2.0], [1e-3, 0.5, 2000.0]])
    oml = np.array([[2e-3, 0.5, 2.0], [2e-3, 0.5, 2000.0]])
    assert band_error(oml, refl) == pytest.approx(3e-6 / 8.0, rel=1e-12)
    # the top band is taken from the reference: a computed top band far off
    # does not move the floor
    assert band_error(np.array([[0.5, 1.0, 1e6]]), ref) > 1e4


def test_all_zero_spectrum_uses_largest_reference_frequency():
    # one plane wave at Gamma: the whole spectrum of that k is zero; it is
    # scaled by the largest reference frequency of the set (3)
    ref = np.array([[0.0, 0.0], [1.0, 3.0]])
    om = np.array([[0.3, 0.0], [1.0, 3.0]])
    assert band_error(om, ref) == pytest.approx(0.09 / 18.0, rel=1e-13)
    # every reference frequency zero: lambda compared against 2
    assert band_error(np.array([[0.2, 0.0]]), np.zeros((1, 2))) == pytest.approx(0.04 / 2.0, rel=1e-13)


def test_shapes():
    with pytest.raises(ValueError):
        band_error(np.zeros((2, 3)), np.zeros((3, 2)))
    # one-dimensional input is one k
    assert band_error(np.array([1.0, 2.2]), np.array([1.0, 2.0])) == pytest.approx(0.1, rel=1e-13)
    assert band_error(np.zeros((0, 3)), np.zeros((0, 3))) == 0.0


def _free_bands(lattice, M, Q, E, nu, rho, nb):
    lam, mu = mo.lame(E, nu)
    cL, cT = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
    A = np.asarray(lattice, dtype=np.float64)
    # reciprocal vectors q^i . h^j = 2 pi delta_ij, from the inverse transpose
    q = 2.0 * np.pi * np.linalg.inv(A).T
    ks = [np.linalg.norm((Q[0] + a) * q[0] + (Q[1] + b) * q[1])
          for a in range(-M, M + 1) for b in range(-M, M + 1)]
    ks = np.array(ks)
    return np.sort(np.concatenate([cL * ks, cT * ks]))[:nb]


@pytest.mark.parametrize("lattice", [np.eye(2), np.array([[1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])])
def test_pwe_homogeneous_cell_is_folded_free_dispersion(lattice):
    """The displacement PWE of a homogeneous cell is exact: c_{L,T} |k + G| for
    the retained plane waves.  This anchors the mixed <= PWE bound: a PWE that
    came out too large would make that bound vacuous."""
    E, nu, rho = 70e9, 0.33, 2700.0
    cell = circle_cell(10, 0.3, inc=(E, nu, rho), mat=(E, nu, rho))
    M, nb = 2, 12
    Qs = np.array([[0.25, 0.1], [0.5, 0.0], [0.31, 0.47]])
    lam = pw.pwe_bands(cell.phase, cell.props, lattice, M, M, Qs, nb)
    for t, Q in enumerate(Qs):
        ref = _free_bands(lattice, M, Q, E, nu, rho, nb)
        assert band_error(np.sqrt(np.maximum(lam[t], 0.0)), ref) < 1e-12
