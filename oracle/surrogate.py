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

Everything is float64 on the CPU: NumPy for the network's bookkeeping and
PyTorch's CPU cross-correlation for the 3x3 convolutions (a library primitive;
the sums it evaluates are written out in conv3x3 / conv3x3_grad).

Optionally (``bf16=True``) the values the network stores are rounded to
bfloat16 where a BF16 implementation stores them: the input channels, the
weights, the hidden activations and the back-propagated output gradients.
The sums themselves stay in float64.  This is the same network evaluated on
BF16-quantised operands, so the rounding decisions, not the arithmetic, are
those of a BF16 kernel.
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


def to_bf16(x):
    """Round to the nearest bfloat16 value, ties to even, returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of an IEEE binary32 value; rounding adds half of the dropped 16-bit field
    (minus one unless the kept field is odd) before truncating.  Values are
    first rounded to binary32.  Non-finite inputs are not expected."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))


def conv3x3(a, W, b=None):
    """Zero-padded 3x3 cross-correlation. a: (B, H, W, Cin), W: (Cout, Cin, 3, 3).

    z[b, y, x, co] = sum_{ci, ky, kx} a[b, y + ky - 1, x + kx - 1, ci] W[co, ci, ky, kx]
    (out-of-range a taken as 0), evaluated in FP64 by the CPU library
    cross-correlation of PyTorch."""
    import torch.nn.functional as F
    z = F.conv2d(_t(a).permute(0, 3, 1, 2), _t(W), padding=1).permute(0, 2, 3, 1).numpy()
    z = np.ascontiguousarray(z)
    if b is not None:
        z += b
    return z


def forward(params, psi, bf16=False):
    """psi: complex (B, H, W).  Returns pred and the cache for backward.
    With bf16, the input channels, weights and hidden activations are
    rounded to bfloat16 (to_bf16) where they are stored."""
    q = to_bf16 if bf16 else (lambda v: v)
    a = q(np.stack([psi.real, psi.imag], axis=-1).astype(np.float64))
    acts, zs = [a], []
    n = len(params)
    for l, (W, b) in enumerate(params):
        z = conv3x3(acts[-1], q(W), b)
        zs.append(z)
        if l < n - 1:
            acts.append(q(np.maximum(z, 0.0)))
    z6 = zs[-1]
    pred = psi + (z6[..., 0] + 1j * z6[..., 1])
    return pred, (acts, zs)


def loss(params, psi, target):
    pred, _ = forward(params, psi)
    d = pred - target
    return float(np.mean(np.concatenate([d.real.ravel(), d.imag.ravel()]) ** 2))


def conv3x3_grad(a, W, dz):
    """Gradients of z = conv3x3(a, W) + b: returns (da, dW, db).

    da[b, y, x, ci] = sum_{co, ky, kx} dz[b, y - ky + 1, x - kx + 1, co] W[co, ci, ky, kx]
    (the cross-correlation of dz with the point-reflected, channel-transposed
    kernel), dW[co, ci, ky, kx] = sum_{b, y, x} dz[b, y, x, co] a[b, y + ky - 1, x + kx - 1, ci],
    db[co] = sum_{b, y, x} dz[b, y, x, co]; FP64, PyTorch CPU library
    correlations."""
    import torch.nn.functional as F
    dzt = _t(dz).permute(0, 3, 1, 2)
    Wt = _t(W)
    da = F.conv2d(dzt, Wt.flip(2, 3).transpose(0, 1), padding=1).permute(0, 2, 3, 1).numpy()
    # dW as the correlation of the input channels with the output gradients,
    # batch folded into the reduction
    at = _t(a).permute(3, 0, 1, 2)           # (Cin, B, H, W)
    dW = F.conv2d(at, dzt.transpose(0, 1), padding=1)  # (Cin, Cout, 3, 3)
    dW = dW.transpose(0, 1).numpy()
    db = np.asarray(dz, dtype=np.float64).sum(axis=(0, 1, 2))
    return np.ascontiguousarray(da), np.ascontiguousarray(dW), db


def loss_and_grad(params, psi, target, bf16=False):
    """MSE loss and its gradient w.r.t. every (W, b), by backpropagation.
    With bf16, forward as above, and the output gradients of every layer are
    rounded to bfloat16 where they are stored; the input gradient of a layer
    is taken with its rounded weights and masked by its rounded activation."""
    q = to_bf16 if bf16 else (lambda v: v)
    pred, (acts, zs) = forward(params, psi, bf16)
    d = pred - target
    nel = 2 * d.size
    dz = q(np.stack([d.real, d.imag], axis=-1) * (2.0 / nel))
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        da, dW, db = conv3x3_grad(acts[l], q(W), dz)
        grads[l] = (dW, db)
        if l > 0:
            dz = q(da * (acts[l] > 0))
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
