"""Pins of the FP64 surrogate reference: central finite differences of the
loss against the hand-written back-propagation, the periodic (circular)
convolution against a direct sum, and exact invariance of the first layer
under circular shifts."""
import numpy as np

from oracle import surrogate_ref as sr


def test_param_count():
    assert sr.n_params() == 262192


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, 8, 8, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    for s in (1, 2):
        z = sr.conv_forward(a, W, b, s)
        ref = np.zeros_like(z)
        for n in range(2):
            for y in range(8 // s):
                for x in range(8 // s):
                    for ky in range(3):
                        for kx in range(3):
                            ref[n, y, x] += a[n, (s * y + ky - 1) % 8, (s * x + kx - 1) % 8] @ W[ky, kx]
        assert np.allclose(z, ref + b, atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    theta = sr.init_params(3)
    # non-zero biases: with zero biases and binary pixels many pre-activations
    # sit exactly on the ReLU kink, where a central difference is not a derivative
    o = 0
    for s in sr.param_shapes():
        n = int(np.prod(s))
        if len(s) == 1:
            theta[o:o + n] = rng.uniform(-0.3, 0.3, n)
        o += n
    x = (rng.uniform(size=(3, 32, 32)) > 0.5).astype(np.float64)
    y = rng.uniform(0.5, 1.5, (3, sr.N_OUT))
    L, g = sr.gradients(theta, x, y)
    assert np.isclose(L, sr.loss(theta, x, y), rtol=1e-14)
    idx = rng.choice(theta.size, 40, replace=False)
    # include entries of every tensor
    starts = np.cumsum([0] + [int(np.prod(s)) for s in sr.param_shapes()])[:-1]
    idx = np.concatenate([idx, starts, starts + 1])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (sr.loss(tp, x, y) - sr.loss(tm, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_first_layer_commutes_with_circular_shift():
    rng = np.random.default_rng(2)
    W = rng.standard_normal((3, 3, 1, 32))
    x = (rng.uniform(size=(1, 32, 32, 1)) > 0.5).astype(float)
    z = sr.conv_forward(x, W, np.zeros(32), 1)
    zs = sr.conv_forward(np.roll(x, (5, -3), axis=(1, 2)), W, np.zeros(32), 1)
    assert np.allclose(np.roll(z, (5, -3), axis=(1, 2)), zs, atol=1e-12)
