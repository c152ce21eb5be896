"""Parity of the eigenvalue sensitivities of the HIP path (through the
C-ABI) against the CPU oracle.

d lambda / d w_f(pixel) = -S^H dPhi S - lambda U^H dOmega U: compared entry
by entry with the oracle's dense per-pixel formula (pinned by finite
differences and Euler's identity on the CPU) on small planar cells of both
layouts; at full size (2N = 882, 18 bands) through Euler's identity, which
holds at any size; on voxel cells against central finite differences of
the three-dimensional oracle.  Bar: 1e-9 of the largest entry per band and
field (FP64), 1e-5 against finite differences.
"""
import numpy as np
import pytest

from oracle import mixed3d_oracle as m3
from oracle import mixed_oracle as mo
from oracle import sensitivity_oracle as so
from synth import config1, random_iso_props, random_voigt_props, voigt_rows_to_matrices

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


def _compare(G, ref):
    """max over (band, field) of the entry error relative to that slice's largest entry."""
    worst = 0.0
    for b in range(ref.shape[0]):
        for f in range(ref.shape[1]):
            scale = np.abs(ref[b, f]).max()
            worst = max(worst, np.abs(G[b, f] - ref[b, f]).max() / scale)
    return worst


@pytest.mark.parametrize("kind", ["anisotropic", "isotropic"])
def test_sensitivities_match_oracle(ctx, kind):
    rng = np.random.default_rng(31)
    phase = rng.integers(0, 3, (6, 5)).astype(np.int32)
    if kind == "anisotropic":
        rows = random_voigt_props(3, rng)
        W, rho = voigt_rows_to_matrices(rows, 2)
        dc = ctx.cell(phase, rows, OBLIQUE)
    else:
        props = random_iso_props(3, rng)
        W, rho = mo.phase_phi_weights(props), props[:, 2]
        dc = ctx.cell(phase, props, OBLIQUE)
    Q = np.array([0.23, 0.11])
    M, nb = 2, 5
    plan = dc.plan(M)
    om, U = plan.solve(Q[None], nb, vectors=True)
    G = plan.sensitivities(Q[None], om, U, phase.shape)[0]
    lam, ref = so.band_sensitivities(phase, W, rho, OBLIQUE, M, M, Q, nb)
    assert np.all(np.diff(lam) > 1e-6 * lam[-1])
    err = _compare(G, ref)
    _say(kind, "sensitivity error", err)
    assert err <= 1e-9


def test_euler_identity_at_full_size(ctx):
    """1132-phase cell at 2N = 882, 18 bands: the compliance sensitivities
    weighted by the compliances, and the density sensitivities weighted by
    the densities, each sum to -lambda (lambda is homogeneous of degree -1
    in each)."""
    c = config1()
    cell = c["cell"]
    W, rho = mo.phase_phi_weights(cell.props), cell.props[:, 2]
    plan = ctx.cell(cell.phase, cell.props).plan(c["M"])
    Q = c["Q"][[7, 33]]
    om, U = plan.solve(Q, c["n_bands"], vectors=True)
    G = plan.sensitivities(Q, om, U, cell.phase.shape)
    pairs = so.field_pairs(3)
    wf = np.stack([W[cell.phase][..., s, t] for s, t in pairs], axis=0)
    lam = om ** 2
    ec = np.einsum("kbfij,fij->kb", G[:, :, :6], wf)
    er = np.einsum("kbij,ij->kb", G[:, :, 6], rho[cell.phase])
    e1, e2 = np.max(np.abs(ec + lam) / lam), np.max(np.abs(er + lam) / lam)
    _say("euler identities", e1, e2)
    assert e1 <= 1e-9 and e2 <= 1e-9


def test_voxel_sensitivities_against_finite_differences(ctx):
    """Anisotropic voxel cell: entries of the GPU sensitivities against central
    differences of the three-dimensional oracle (the voxel given its own
    phase), and Euler's identity."""
    rng = np.random.default_rng(32)
    phase = rng.integers(0, 2, (3, 3, 2)).astype(np.int32)
    rows = random_voigt_props(2, rng, dim=3)
    W, rho = voigt_rows_to_matrices(rows, 3)
    Q = np.array([0.21, -0.13, 0.34])
    M, nb = 1, 4
    plan = ctx.cell_voxels(phase, rows).plan(M)
    om, U = plan.solve(Q[None], nb, vectors=True)
    G = plan.sensitivities(Q[None], om, U, phase.shape)[0]     # [nb, 22, 3, 3, 2]
    lam = om[0] ** 2
    iu = np.triu_indices(6)
    wf = np.stack([W[phase][..., s, t] for s, t in zip(*iu)], axis=0)
    ec = np.einsum("bfijk,fijk->b", G[:, :21], wf)
    er = np.einsum("bijk,ijk->b", G[:, 21], rho[phase])
    assert np.max(np.abs(ec + lam) / lam) <= 1e-9 and np.max(np.abs(er + lam) / lam) <= 1e-9
    pairs = list(zip(*iu))
    for (i, j, k), f in [((0, 1, 1), 0), ((2, 0, 0), 5), ((1, 2, 1), 21), ((1, 1, 0), 15)]:
        p0 = phase[i, j, k]
        out = []
        for sign in (1.0, -1.0):
            ph = phase.copy()
            ph[i, j, k] = 2
            W2 = np.concatenate([W, W[p0:p0 + 1]], axis=0)
            r2 = np.concatenate([rho, rho[p0:p0 + 1]])
            if f < 21:
                s, t = pairs[f]
                h = 1e-6 * W[p0, s, s]
                W2[2, s, t] += sign * h
                if s != t:
                    W2[2, t, s] += sign * h
            else:
                h = 1e-6 * rho[p0]
                r2[2] += sign * h
            props = np.stack([np.ones(3), np.zeros(3), r2], axis=1)
            _, l2 = m3.bands3(ph, props, np.eye(3), M, M, M, Q[None], nb, weights=W2)
            out.append(l2[0])
        fd = (out[0] - out[1]) / (2 * h)
        scale = np.abs(G[:, f]).reshape(nb, -1).max(axis=1)
        err = np.max(np.abs(G[:, f, i, j, k] - fd) / scale)
        _say("voxel fd", (i, j, k), f, err)
        assert err <= 1e-5
