"""Pins of the corrector oracle against what the definitions fix: finite
differences of the loss, numpy's correlate, exact shifts, positive
homogeneity and Adam's closed-form first step."""
import numpy as np
import pytest

from oracle import corrector as oc


def _rand(seed, c_in=3, c_out=2, B=2, J=11, scale=0.3):
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, scale, oc.num_weights(c_in, c_out))
    x = rng.normal(0.0, 1.0, (B, c_in, J))
    t = rng.normal(0.0, 1.0, (B, c_out, J))
    return w, x, t


def test_weight_count():
    # 5 * (c_in*32 + 32*32 + 32*32 + 32*c_out)
    assert oc.num_weights(8, 4) == 5 * (8 * 32 + 32 * 32 * 2 + 32 * 4)


def test_single_channel_conv_is_numpy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 1, 9))
    W = rng.normal(size=(1, 1, 5))
    y = oc.conv1d(x, W)
    ref = np.correlate(np.pad(x[0, 0], 2), W[0, 0], mode="valid")
    np.testing.assert_allclose(y[0, 0], ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("tap,shift", [(0, -2), (1, -1), (2, 0), (3, 1), (4, 2)])
def test_delta_kernel_shifts_with_zero_fill(tap, shift):
    # W[o, i, t] = delta(o, i) delta(t, tap): y[j] = x[j + tap - 2], zero past the ends
    x = np.arange(1.0, 8.0).reshape(1, 1, 7) * np.array([1.0, -2.0]).reshape(1, 2, 1)
    W = np.zeros((2, 2, 5))
    W[0, 0, tap] = W[1, 1, tap] = 1.0
    y = oc.conv1d(x, W)
    for c in range(2):
        for j in range(7):
            k = j + shift
            assert y[0, c, j] == (x[0, c, k] if 0 <= k < 7 else 0.0)


def test_positive_homogeneity():
    w, x, _ = _rand(2)
    y1, _ = oc.forward(w, x, 3, 2)
    y2, _ = oc.forward(w, 3.5 * x, 3, 2)
    np.testing.assert_allclose(y2, 3.5 * y1, rtol=1e-13, atol=1e-13)


def test_relu_zeroes_negative_hidden_values():
    w, x, _ = _rand(3)
    _, acts = oc.forward(w, x, 3, 2)
    for h in acts[1:-1]:
        assert h.min() >= 0.0 and (h == 0.0).any()


@pytest.mark.parametrize("seed", [4, 5])
def test_gradient_matches_central_differences(seed):
    w, x, t = _rand(seed)
    L, g = oc.grad(w, x, t, 3, 2)
    assert L == pytest.approx(oc.loss(w, x, t, 3, 2), rel=1e-15)
    rng = np.random.default_rng(seed + 100)
    idx = rng.choice(w.size, 40, replace=False)
    # every layer's first and last weight as well
    bounds = np.cumsum([0] + [int(np.prod(s)) for s in oc.layer_shapes(3, 2)])
    idx = np.unique(np.concatenate([idx, bounds[:-1], bounds[1:] - 1]))
    h = 1e-6
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (oc.loss(wp, x, t, 3, 2) - oc.loss(wm, x, t, 3, 2)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9), k


def test_adam_first_step_closed_form():
    # t = 1: m_hat = g, v_hat = g^2, so w moves by lr * g / (|g| + eps)
    rng = np.random.default_rng(6)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    w1, m, v = oc.adam(w, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_moves_by_lr_each_step():
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    w = np.array([1.0, -2.0])
    g = np.array([0.5, -4.0])
    m = v = np.zeros(2)
    for t in range(1, 6):
        w, m, v = oc.adam(w, g, m, v, t, 0.01, eps=0.0)
    np.testing.assert_allclose(w, np.array([1.0, -2.0]) - 5 * 0.01 * np.sign(g), rtol=1e-12)
