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
