"""CPU checks of the surrogate's full-size parity criteria
(tests/surrogate_criteria.py): an FP32 emulation of the GPU's roundings (BF16
operands, FP32 sums, BF16 stores at the same points) meets them, and planted
mistakes of the kinds the GPU kernels could make do not.  The emulation uses
PyTorch's CPU FP32 correlations; it is test infrastructure, not a model of
the kernels' summation order."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import surrogate as S
from paper_1203_1263_amd import workloads as wl
from surrogate_criteria import SURROGATE_CRITERIA, bf16_forward_with_scale, bf16_grads_with_scales, worst_ratio

q = S.to_bf16


def _c32(a, W, b=None):
    import torch
    import torch.nn.functional as F
    z = F.conv2d(torch.from_numpy(a.astype(np.float32)).permute(0, 3, 1, 2),
                 torch.from_numpy(W.astype(np.float32)), padding=1).permute(0, 2, 3, 1).numpy()
    if b is not None:
        z = (z + b.astype(np.float32)).astype(np.float32)
    return z


def _c32_t(dz, W):
    import torch
    import torch.nn.functional as F
    return F.conv2d(torch.from_numpy(dz.astype(np.float32)).permute(0, 3, 1, 2),
                    torch.from_numpy(W.astype(np.float32)).flip(2, 3).transpose(0, 1),
                    padding=1).permute(0, 2, 3, 1).numpy()


def _wgrad32(a, dz):
    import torch
    import torch.nn.functional as F
    at = torch.from_numpy(a.astype(np.float32)).permute(3, 0, 1, 2)
    dt = torch.from_numpy(dz.astype(np.float32)).permute(3, 0, 1, 2)
    return F.conv2d(at, dt, padding=1).transpose(0, 1).numpy().astype(np.float64)


def emulate(p, x, t):
    """Forward output and gradients with BF16 operands and FP32 sums."""
    acts = [q(np.stack([x.real, x.imag], axis=-1))]
    for l, (W, b) in enumerate(p):
        z = _c32(acts[-1], q(W), b)
        if l < len(p) - 1:
            acts.append(q(np.maximum(z, 0.0)))
    pr = (x.real.astype(np.float32) + z[..., 0]).astype(np.float64)
    pi = (x.imag.astype(np.float32) + z[..., 1]).astype(np.float64)
    pred = pr + 1j * pi
    d = np.stack([(pr - t.real).astype(np.float32), (pi - t.imag).astype(np.float32)], axis=-1)
    dz = q(d.astype(np.float64) * (2.0 / d.size))
    grads = [None] * len(p)
    for l in range(len(p) - 1, -1, -1):
        grads[l] = [_wgrad32(acts[l], dz), dz.astype(np.float32).sum(axis=(0, 1, 2)).astype(np.float64)]
        if l > 0:
            dz = q(_c32_t(dz, q(p[l][0])) * (acts[l] > 0))
    return pred, grads


def _case(H=64, W=64, B=2):
    g = np.random.Generator(np.random.PCG64(31))
    x = np.array([wl.surrogate_ic(g, n=256, h=0.25)[96:96 + H, 96:96 + W] for _ in range(B)])
    x = x.astype(np.complex64).astype(np.complex128)
    t = (x * np.exp(-0.15j) + 0.05 * x.conj()).astype(np.complex64).astype(np.complex128)
    p = S.unpack(S.pack(S.init_params(32)).astype(np.float32).astype(np.float64))
    return p, x, t


def _fails(p, x, pred, grads, t):
    """Which criteria a candidate (pred, grads) breaks."""
    out = []
    rb, (sr, si) = bf16_forward_with_scale(p, x)
    if max(worst_ratio(pred.real, rb.real, sr), worst_ratio(pred.imag, rb.imag, si)) > 1.0:
        out.append("fwd_elem")
    if np.linalg.norm(pred - rb) / np.linalg.norm(rb - x) >= SURROGATE_CRITERIA["bf16_norm"]:
        out.append("fwd_norm")
    _, gr, sc = bf16_grads_with_scales(p, x, t)
    for l in range(len(p)):
        for k, name in ((0, "W"), (1, "b")):
            if worst_ratio(grads[l][k], gr[l][k], sc[l][k]) > 1.0:
                out.append(f"elem{name}{l + 1}")
            if np.linalg.norm(grads[l][k] - gr[l][k]) / np.linalg.norm(gr[l][k]) >= SURROGATE_CRITERIA["bf16_norm"]:
                out.append(f"norm{name}{l + 1}")
    return out


@pytest.fixture(scope="module")
def case():
    p, x, t = _case()
    pred, grads = emulate(p, x, t)
    return p, x, t, pred, grads


def test_fp32_emulation_meets_the_criteria(case):
    p, x, t, pred, grads = case
    assert _fails(p, x, pred, grads, t) == []


def test_planted_transposed_taps_fail(case):
    p, x, t, pred, grads = case
    bad = [list(g) for g in grads]
    bad[2][0] = bad[2][0].transpose(0, 1, 3, 2).copy()  # ky <-> kx in layer 3
    assert any(f.endswith("W3") for f in _fails(p, x, pred, bad, t))


def test_planted_dropped_tile_fails(case):
    """One 16 x 8 pixel tile of the 64 left out of layer 4's weight gradient."""
    p, x, t, pred, grads = case
    # layer 4's output gradient from the reference's backward pass
    pr, (racts, _) = S.forward(p, x, bf16=True)
    d = pr - t
    dz = q(np.stack([d.real, d.imag], axis=-1) * (2.0 / (2 * d.size)))
    for l in range(len(p) - 1, 3, -1):
        da, _, _ = S.conv3x3_grad(racts[l], q(p[l][0]), dz)
        dz = q(da * (racts[l] > 0))
    dz_tile = np.zeros_like(dz)
    dz_tile[0, 8:16, 16:32] = dz[0, 8:16, 16:32]
    _, dW_tile, db_tile = S.conv3x3_grad(racts[3], q(p[3][0]), dz_tile)
    bad = [list(g) for g in grads]
    bad[3][0] = bad[3][0] - dW_tile
    bad[3][1] = bad[3][1] - db_tile
    assert "normW4" in _fails(p, x, pred, bad, t)


def test_planted_shifted_output_tile_fails(case):
    """One 16 x 16 output tile taken one pixel to the left."""
    p, x, t, pred, grads = case
    bad = pred.copy()
    bad[1, 16:32, 17:32] = pred[1, 16:32, 16:31]
    assert "fwd_elem" in _fails(p, x, bad, grads, t)
