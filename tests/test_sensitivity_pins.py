"""Pins of the eigenvalue-sensitivity oracle (no GPU).

The oracle writes d lambda = -S^H dPhi S - lambda U^H dOmega U out densely,
one pixel at a time.  Two facts fix it independently of that formula:
central finite differences of the band oracle with the pixel given a phase
of its own, and Euler's identity: lambda is homogeneous of degree -1 in the
compliance weights (A = H Phi^-1 H*) and of degree -1 in the density
(Omega), so sum_p sum_f w_f(p) d lambda / d w_f(p) = -lambda for each.
A dropped mirror block, a wrong sign or a missing lambda factor fails one of
them.
"""
import numpy as np
import pytest

from oracle import sensitivity_oracle as so
from synth import random_voigt_props, voigt_rows_to_matrices

OBLIQUE = np.array([[1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])


def _cell(seed, shape=(4, 3), P=2):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, P, shape).astype(np.int32)
    W, rho = voigt_rows_to_matrices(random_voigt_props(P, rng), 2)
    return phase, W, rho


@pytest.mark.parametrize("lattice", [np.eye(2), OBLIQUE])
def test_sensitivities_match_finite_differences(lattice):
    phase, W, rho = _cell(3)
    Q = np.array([0.23, 0.11])
    M, nb = 2, 4
    lam, G = so.band_sensitivities(phase, W, rho, lattice, M, M, Q, nb)
    assert np.all(np.diff(lam) > 1e-6 * lam[-1])            # simple eigenvalues
    for pixel in [(0, 0), (2, 1), (3, 2)]:
        for f in range(7):
            fd = so.finite_difference(phase, W, rho, lattice, M, M, Q, nb, pixel, f)
            scale = np.abs(G[:, f]).max(axis=(1, 2))
            err = np.abs(G[:, f, pixel[0], pixel[1]] - fd) / scale
            assert np.all(err < 2e-5), (pixel, f, err)


def test_euler_identity_for_compliance_and_density():
    phase, W, rho = _cell(4, (5, 4), 3)
    Q = np.array([0.4, -0.17])
    lam, G = so.band_sensitivities(phase, W, rho, OBLIQUE, 2, 1, Q, 6)
    pairs = so.field_pairs(3)
    wf = np.stack([W[phase][..., s, t] for s, t in pairs], axis=0)     # [6, nx, ny]
    euler_c = np.einsum("bfij,fij->b", G[:, :6], wf)
    euler_r = np.einsum("bij,ij->b", G[:, 6], rho[phase])
    assert np.allclose(euler_c, -lam, rtol=1e-10, atol=0)
    assert np.allclose(euler_r, -lam, rtol=1e-10, atol=0)


def test_uniform_scaling_of_one_field_is_the_field_sum():
    """Moving a field of every pixel of phase p by the same amount is moving
    that phase's weight: the sum of the pixel sensitivities over the phase
    equals the finite difference of the phase weight."""
    phase, W, rho = _cell(5)
    Q = np.array([0.31, 0.05])
    lam, G = so.band_sensitivities(phase, W, rho, np.eye(2), 2, 2, Q, 3)
    f, (s, t) = 4, so.field_pairs(3)[4]
    h = 1e-6 * abs(W[0, s, s])
    from oracle import mixed_oracle as mo
    import scipy.linalg as sla
    out = []
    for sign in (1.0, -1.0):
        W2 = W.copy()
        W2[0, s, t] += sign * h
        W2[0, t, s] += sign * h
        props = np.stack([np.ones(2), np.zeros(2), rho], axis=1)
        I = mo.subdomain_integral_tables(phase, 2, np.eye(2), 2, 2)
        mats = mo.assemble(I, props, np.eye(2), 2, 2, Q, tables=mo.phase_sum_tables(I, props, phase_weights=W2))
        out.append(sla.eigh(mo.reduced_operator(mats), mats["Omega"], eigvals_only=True, subset_by_index=[0, 2]))
    fd = (out[0] - out[1]) / (2 * h)
    tot = np.array([G[b, f][phase == 0].sum() for b in range(3)])
    assert np.allclose(tot, fd, rtol=1e-5)
