"""FP64 NumPy reference of the band-structure surrogate network (test infrastructure).

TEST INFRASTRUCTURE ONLY (see mixed_oracle).  The network the GPU library
trains and runs, written out plainly so that its forward pass and gradients
can be checked:

  input   x [B, 32, 32, 1]   binary pixel cell (NHWC)
  conv1   3x3, 1 -> 32,  stride 1, circular padding, ReLU   -> [B, 32, 32, 32]
  conv2   3x3, 32 -> 32, stride 2, circular padding, ReLU   -> [B, 16, 16, 32]
  conv3   3x3, 32 -> 32, stride 2, circular padding, ReLU   -> [B,  8,  8, 32]
  conv4   3x3, 32 -> 32, stride 2, circular padding, ReLU   -> [B,  4,  4, 32]
  flatten (y, x, c) -> 512
  fc1     512 -> 256, ReLU
  fc2     256 -> 400   (10 bands x 40 k-points, normalised frequencies)
  loss    mean squared error over all outputs

Circular padding makes the convolution periodic like the unit cell: output
pixel (y, x) of a stride-s layer reads input pixels ((s y + ky - 1) mod H,
(s x + kx - 1) mod W), ky, kx in 0..2.  Parameters are one flat vector in the
order conv1 W, b, conv2 W, b, conv3 W, b, conv4 W, b, fc1 W, b, fc2 W, b;
conv weights are laid out [ky][kx][ci][co], fully connected ones [in][out].
"""
from __future__ import annotations

import numpy as np

CONV = [(1, 32, 1), (32, 32, 2), (32, 32, 2), (32, 32, 2)]   # (ci, co, stride)
FC = [(512, 256), (256, 400)]
N_OUT = 400


def param_shapes():
    shapes = []
    for ci, co, _ in CONV:
        shapes += [(3, 3, ci, co), (co,)]
    for a, b in FC:
        shapes += [(a, b), (b,)]
    return shapes


def n_params():
    return int(sum(np.prod(s) for s in param_shapes()))


def unflatten(theta):
    out, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def init_params(seed):
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in param_shapes():
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[:-1]))
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, s))
    return np.concatenate([p.ravel() for p in parts])


def _taps(H, W, s):
    """Input row/column index of every output pixel for each kernel tap."""
    Ho, Wo = H // s, W // s
    iy = [(s * np.arange(Ho) + ky - 1) % H for ky in range(3)]
    ix = [(s * np.arange(Wo) + kx - 1) % W for kx in range(3)]
    return iy, ix


def conv_forward(a, Wt, b, s):
    B, H, W, ci = a.shape
    iy, ix = _taps(H, W, s)
    z = np.zeros((B, H // s, W // s, Wt.shape[3]))
    for ky in range(3):
        for kx in range(3):
            patch = a[:, iy[ky]][:, :, ix[kx]]                   # [B, Ho, Wo, ci]
            z += patch @ Wt[ky, kx]
    return z + b


def conv_backward(a, Wt, dz, s):
    """Gradients of z = conv(a) with respect to a, W and b."""
    B, H, W, ci = a.shape
    iy, ix = _taps(H, W, s)
    da = np.zeros_like(a)
    dW = np.zeros_like(Wt)
    for ky in range(3):
        for kx in range(3):
            patch = a[:, iy[ky]][:, :, ix[kx]]
            dW[ky, kx] = np.tensordot(patch, dz, axes=([0, 1, 2], [0, 1, 2]))
            contrib = dz @ Wt[ky, kx].T                          # [B, Ho, Wo, ci]
            # for a fixed tap every output pixel reads a distinct input pixel
            da[:, iy[ky][:, None], ix[kx][None, :]] += contrib
    db = dz.sum(axis=(0, 1, 2))
    return da, dW, db


def forward(theta, x, keep=False):
    p = unflatten(np.asarray(theta, dtype=np.float64))
    a = np.asarray(x, dtype=np.float64).reshape(-1, 32, 32, 1)
    acts = [a]
    for li, (_, _, s) in enumerate(CONV):
        a = np.maximum(conv_forward(a, p[2 * li], p[2 * li + 1], s), 0.0)
        acts.append(a)
    f = a.reshape(a.shape[0], -1)
    h = np.maximum(f @ p[8] + p[9], 0.0)
    out = h @ p[10] + p[11]
    if keep:
        return out, (acts, f, h)
    return out


def loss(theta, x, y):
    out = forward(theta, x)
    return float(np.mean((out - y) ** 2))


def gradients(theta, x, y):
    """(loss, d loss / d theta) by hand-written back-propagation."""
    p = unflatten(np.asarray(theta, dtype=np.float64))
    out, (acts, f, h) = forward(theta, x, keep=True)
    y = np.asarray(y, dtype=np.float64).reshape(out.shape)
    L = float(np.mean((out - y) ** 2))
    dout = 2.0 * (out - y) / out.size
    g = [None] * 12
    g[10] = h.T @ dout
    g[11] = dout.sum(axis=0)
    dh = (dout @ p[10].T) * (h > 0)
    g[8] = f.T @ dh
    g[9] = dh.sum(axis=0)
    da = (dh @ p[8].T).reshape(acts[-1].shape)
    for li in range(3, -1, -1):
        _, _, s = CONV[li]
        dz = da * (acts[li + 1] > 0)
        da, g[2 * li], g[2 * li + 1] = conv_backward(acts[li], p[2 * li], dz, s)
    return L, np.concatenate([t.ravel() for t in g])
