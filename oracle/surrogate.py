"""FP64 CPU reference of the convolutional surrogate (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by tests and the smoke check to verify the
GPU surrogate kernels; never imported by the product path.

The network (not part of the paper; it is the learned surrogate the GPU
library trains on the integrator's own trajectories) maps a complex field
psi (stored as 2 real channels, re and im) to psi + net(psi):

    a0 = [Re psi, Im psi]                       (H x W x 2)
    z_l = conv3x3(a_{l-1}, W_l) + b_l           l = 1..6, zero "same" padding
    a_l = relu(z_l)                             l = 1..5
    pred = psi + (z_6[..., 0] + i z_6[..., 1])

Channels 2 -> 48 -> 48 -> 48 -> 48 -> 48 -> 2.  W_l has shape
(C_out, C_in, 3, 3) and conv3x3 is a cross-correlation:
z[y, x, co] = sum_{ci, ky, kx} a[y + ky - 1, x + kx - 1, ci] W[co, ci, ky, kx].
Loss: mean over batch, pixels and the 2 channels of (pred - target)^2.

Everything is plain NumPy in float64, written for clarity, not speed.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 48, 48, 48, 48, 48, 2)


def param_shapes(channels=CHANNELS):
    out = []
    for l in range(len(channels) - 1):
        out.append(((channels[l + 1], channels[l], 3, 3), (channels[l + 1],)))
    return out


def param_count(channels=CHANNELS) -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes(channels))


def unpack(flat, channels=CHANNELS):
    """Flat parameter vector -> list of (W, b); order W1, b1, W2, b2, ..."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for ws, bs in param_shapes(channels):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((flat[o:o + nw].reshape(ws), flat[o + nw:o + nw + nb].reshape(bs)))
        o += nw + nb
    assert o == flat.size
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def conv3x3(a, W, b=None):
    """Zero-padded 3x3 cross-correlation. a: (B, H, W, Cin), W: (Cout, Cin, 3, 3)."""
    Bn, H, Wd, _ = a.shape
    ap = np.zeros((Bn, H + 2, Wd + 2, a.shape[3]))
    ap[:, 1:-1, 1:-1, :] = a
    z = np.zeros((Bn, H, Wd, W.shape[0]))
    for ky in range(3):
        for kx in range(3):
            z += ap[:, ky:ky + H, kx:kx + Wd, :] @ W[:, :, ky, kx].T
    if b is not None:
        z += b
    return z


def forward(params, psi):
    """psi: complex (B, H, W).  Returns pred and the cache for backward."""
    a = np.stack([psi.real, psi.imag], axis=-1).astype(np.float64)
    acts, zs = [a], []
    n = len(params)
    for l, (W, b) in enumerate(params):
        z = conv3x3(acts[-1], W, b)
        zs.append(z)
        if l < n - 1:
            acts.append(np.maximum(z, 0.0))
    z6 = zs[-1]
    pred = psi + (z6[..., 0] + 1j * z6[..., 1])
    return pred, (acts, zs)


def loss(params, psi, target):
    pred, _ = forward(params, psi)
    d = pred - target
    return float(np.mean(np.concatenate([d.real.ravel(), d.imag.ravel()]) ** 2))


def conv3x3_grad(a, W, dz):
    """Gradients of z = conv3x3(a, W) + b: returns (da, dW, db)."""
    Bn, H, Wd, Cin = a.shape
    ap = np.zeros((Bn, H + 2, Wd + 2, Cin))
    ap[:, 1:-1, 1:-1, :] = a
    dW = np.zeros_like(W)
    dap = np.zeros_like(ap)
    for ky in range(3):
        for kx in range(3):
            win = ap[:, ky:ky + H, kx:kx + Wd, :]
            dW[:, :, ky, kx] = np.einsum("bhwo,bhwi->oi", dz, win)
            dap[:, ky:ky + H, kx:kx + Wd, :] += dz @ W[:, :, ky, kx]
    db = dz.sum(axis=(0, 1, 2))
    return dap[:, 1:-1, 1:-1, :], dW, db


def loss_and_grad(params, psi, target):
    """MSE loss and its gradient w.r.t. every (W, b), by backpropagation."""
    pred, (acts, zs) = forward(params, psi)
    d = pred - target
    nel = 2 * d.size
    dz = np.stack([d.real, d.imag], axis=-1) * (2.0 / nel)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        da, dW, db = conv3x3_grad(acts[l], W, dz)
        grads[l] = (dW, db)
        if l > 0:
            dz = da * (zs[l - 1] > 0)
    L = float(np.mean(np.concatenate([d.real.ravel(), d.imag.ravel()]) ** 2))
    return L, grads


def init_params(seed: int, channels=CHANNELS, last_scale: float = 0.1):
    """He-normal initial weights (last layer scaled down), zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for l, (ws, bs) in enumerate(param_shapes(channels)):
        fan_in = ws[1] * 9
        W = g.standard_normal(ws) * np.sqrt(2.0 / fan_in)
        if l == len(channels) - 2:
            W *= last_scale
        out.append((W, np.zeros(bs)))
    return out


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Textbook Adam (Kingma & Ba) on flat FP64 arrays; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
