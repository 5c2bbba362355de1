"""Pins of the FP64 CPU reference of the convolutional surrogate."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import surrogate as S


def test_param_count():
    # 2->48, 4 x 48->48, 48->2, 3x3 kernels with biases
    assert S.param_count() == (48 * 2 * 9 + 48) + 4 * (48 * 48 * 9 + 48) + (2 * 48 * 9 + 2) == 84914


def test_conv_matches_scipy_correlate():
    g = np.random.default_rng(0)
    a = g.standard_normal((2, 7, 9, 3))
    W = g.standard_normal((4, 3, 3, 3))
    b = g.standard_normal(4)
    z = S.conv3x3(a, W, b)
    for bi in range(2):
        for co in range(4):
            ref = sum(correlate2d(a[bi, :, :, ci], W[co, ci], mode="same", boundary="fill") for ci in range(3))
            assert np.allclose(z[bi, :, :, co], ref + b[co], atol=1e-12)


def test_zero_last_layer_is_identity():
    p = S.init_params(1)
    W6, b6 = p[-1]
    p[-1] = (np.zeros_like(W6), np.zeros_like(b6))
    psi = np.exp(1j * np.linspace(0, 3, 64)).reshape(1, 8, 8)
    pred, _ = S.forward(p, psi)
    assert np.array_equal(pred, psi)


def test_gradients_match_central_differences():
    ch = (2, 5, 4, 2)
    g = np.random.default_rng(3)
    params = [(g.standard_normal(w) * 0.4, g.standard_normal(b) * 0.1) for w, b in S.param_shapes(ch)]
    psi = g.standard_normal((2, 6, 7)) + 1j * g.standard_normal((2, 6, 7))
    tgt = g.standard_normal((2, 6, 7)) + 1j * g.standard_normal((2, 6, 7))
    L, grads = S.loss_and_grad(params, psi, tgt)
    flat = S.pack(params)
    gflat = S.pack(grads)
    idx = g.choice(flat.size, 40, replace=False)
    eps = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += eps
        fm[i] -= eps
        num = (S.loss(S.unpack(fp, ch), psi, tgt) - S.loss(S.unpack(fm, ch), psi, tgt)) / (2 * eps)
        assert num == pytest.approx(gflat[i], rel=1e-5, abs=1e-9)
    assert L == pytest.approx(S.loss(params, psi, tgt), rel=1e-14)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = S.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)


def test_conv_gradients_match_scipy_and_loops():
    """The input gradient is the full correlation of dz with the point-
    reflected kernel (a 'same' convolution), the weight gradient the plain
    sum of dz times the shifted, zero-padded input."""
    from scipy.signal import convolve2d
    g = np.random.default_rng(4)
    a = g.standard_normal((2, 6, 5, 3))
    W = g.standard_normal((4, 3, 3, 3))
    dz = g.standard_normal((2, 6, 5, 4))
    da, dW, db = S.conv3x3_grad(a, W, dz)
    for bi in range(2):
        for ci in range(3):
            ref = sum(convolve2d(dz[bi, :, :, co], W[co, ci], mode="same") for co in range(4))
            assert np.allclose(da[bi, :, :, ci], ref, atol=1e-12)
    ap = np.zeros((2, 8, 7, 3))
    ap[:, 1:-1, 1:-1] = a
    for co in range(4):
        for ci in range(3):
            for ky in range(3):
                for kx in range(3):
                    ref = np.sum(dz[:, :, :, co] * ap[:, ky:ky + 6, kx:kx + 5, ci])
                    assert dW[co, ci, ky, kx] == pytest.approx(ref, abs=1e-12)
    assert np.allclose(db, dz.sum(axis=(0, 1, 2)), atol=1e-12)


def test_bf16_rounding_matches_torch_and_ties_to_even():
    """to_bf16 against PyTorch's own float32 -> bfloat16 conversion, plus
    hand-checked ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and goes
    to the even 1; 1 + 3 * 2^-8 goes up to the even 1 + 2^-6."""
    import torch
    g = np.random.default_rng(7)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.integers(-20, 20, 20000),
                        [0.0, -0.0, 1.0, -2.5, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.to_bf16(x), ref)
    assert S.to_bf16(1 + 2.0 ** -8) == 1.0
    assert S.to_bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6


def test_bf16_mode_is_the_same_network_on_rounded_operands():
    """With every stored value already a bfloat16 number the BF16 mode
    changes nothing; on general inputs it differs from FP64 by about the
    BF16 unit roundoff."""
    p = S.init_params(3, channels=(2, 6, 6, 2))
    g = np.random.default_rng(8)
    psi = g.standard_normal((2, 9, 7)) + 1j * g.standard_normal((2, 9, 7))
    pr, _ = S.forward(p, psi)
    pb, _ = S.forward(p, psi, bf16=True)
    inc = pr - psi
    err = np.linalg.norm(pb - pr) / np.linalg.norm(inc)
    assert 1e-4 < err < 3e-2
    # a network whose hidden activations are exactly representable: one layer
    p1 = [(S.to_bf16(p[0][0][:2]), np.zeros(2))]
    psi_b = S.to_bf16(psi.real) + 1j * S.to_bf16(psi.imag)
    a, _ = S.forward(p1, psi_b)
    b, _ = S.forward(p1, psi_b, bf16=True)
    assert np.array_equal(a, b)
