"""Parity criteria of the surrogate's full-size GPU tests against the
BF16-mode FP64 reference (oracle/surrogate.py), kept apart so a CPU test can
check them on an FP32 emulation of the GPU's roundings and on planted
mistakes.  The derivation is stated in tests/test_gpu_surrogate.py."""
from __future__ import annotations

import numpy as np

from oracle import surrogate as S

# one BF16 unit in the last place relative to the value (2u, u = 2^-8), and
# the normwise bar against the BF16-mode reference
SURROGATE_CRITERIA = {"ulp": 2.0 ** -7, "bf16_norm": 2e-3}


def _wgrad_abs(a, g):
    """Sum over pixels of |g[p, co]| |a[p + tap, ci]| (the magnitudes of the
    weight-gradient terms), FP64."""
    import torch
    import torch.nn.functional as F
    at = torch.from_numpy(np.ascontiguousarray(np.abs(a))).permute(3, 0, 1, 2)
    gt = torch.from_numpy(np.ascontiguousarray(np.abs(g))).permute(3, 0, 1, 2)
    return F.conv2d(at, gt, padding=1).transpose(0, 1).numpy()


def _g32(k):
    """Bound factor of an FP32 sum of k terms: k u32 / (1 - k u32)."""
    return k * 2.0 ** -24 / (1.0 - k * 2.0 ** -24)


def _forward_with_allowances(p, x):
    """BF16-mode forward pass plus, per layer, the band within which the
    GPU's FP32 pre-activation may differ from the reference's (g(K) times
    the sum of the magnitudes of its terms) and the allowance of every
    stored activation (one BF16 ulp, 2u of the value, plus that band)."""
    q = S.to_bf16
    pred, (acts, zs) = S.forward(p, x, bf16=True)
    c = SURROGATE_CRITERIA["ulp"]
    band, ea = [], [np.zeros_like(acts[0])]  # the input channels are rounded alike
    for l, (W, b) in enumerate(p):
        M = S.conv3x3(np.abs(acts[l]), np.abs(q(W)), np.abs(b))
        band.append(_g32(9 * W.shape[1] + 1) * M)
        if l < len(p) - 1:
            ea.append(c * np.abs(acts[l + 1]) + band[-1])
    return pred, acts, zs, band, ea


def bf16_forward_with_scale(p, x):
    """BF16-mode forward pass and the element-wise bound of every output:
    the last layer's terms with their activation allowances, its own FP32
    band, and the FP32 rounding of the stored output."""
    rb, acts, zs, band, ea = _forward_with_allowances(p, x)
    W6, _ = p[-1]
    e6 = S.conv3x3(ea[-1], np.abs(S.to_bf16(W6))) + band[-1]
    return rb, (e6[..., 0] + 2.0 ** -23 * np.abs(rb.real), e6[..., 1] + 2.0 ** -23 * np.abs(rb.imag))


def bf16_grads_with_scales(p, x, t):
    """The reference's BF16-mode backpropagation and, for every layer, the
    element-wise bounds of its weight and bias gradients.  A term
    dz[p, co] a[p + tap, ci] may differ through either operand: a by its
    forward allowance, dz by one BF16 ulp (2u of its value) and, where the
    ReLU of its pre-activation is undecided (|z| within the FP32 band), by
    the whole back-propagated value."""
    q = S.to_bf16
    pred, acts, zs, band, ea = _forward_with_allowances(p, x)
    d = pred - t
    scale = 2.0 / (2 * d.size)
    dz = q(np.stack([d.real, d.imag], axis=-1) * scale)
    c = SURROGATE_CRITERIA["ulp"]
    edz = c * np.abs(dz) + scale * (band[-1] + 2.0 ** -23 * np.abs(np.stack([pred.real, pred.imag], axis=-1)))
    scales = [None] * len(p)
    for l in range(len(p) - 1, -1, -1):
        W, _ = p[l]
        da, _, _ = S.conv3x3_grad(acts[l], q(W), dz)
        a_abs = np.abs(acts[l])
        kw = 4096  # pixels one FP32 gradient partial may sum
        eW = _wgrad_abs(a_abs, edz) + _wgrad_abs(ea[l], np.abs(dz)) + _g32(kw) * _wgrad_abs(a_abs, dz)
        eb = edz.sum(axis=(0, 1, 2)) + _g32(kw) * np.abs(dz).sum(axis=(0, 1, 2))
        # differences that enter through the shared output gradient dz[., co]
        # (propagated from the layers above) are not local to one element:
        # every element of output channel co gets the largest first-order
        # bound of that channel
        rowmax = eW.reshape(eW.shape[0], -1).max(axis=1)
        scales[l] = (np.broadcast_to(rowmax[:, None, None, None], eW.shape).copy(), eb)
        if l > 0:
            undecided = np.abs(zs[l - 1]) <= band[l - 1]
            dz = q(da * (acts[l] > 0))
            edz = c * np.abs(dz) + np.where(undecided, np.abs(da), 0.0)
    L, grads = S.loss_and_grad(p, x, t, bf16=True)
    return L, grads, scales


def worst_ratio(got, ref, scale):
    """Largest |got - ref| / scale over the elements (0/0 counts as 0)."""
    diff = np.abs(got - ref)
    return float(np.max(np.where(diff == 0, 0.0, diff / np.maximum(scale, 1e-300))))
