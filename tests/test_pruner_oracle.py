"""Pins of the pruner's FP64 oracle (CPU only): finite differences, closed
forms, a hand-worked forward pass, Adam's first step, the keep rule."""

import math

import numpy as np
import pytest

import kgsynth
from oracle import pruner as P


def _net(d, H, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.normal(0.0, 0.6, P.param_count(d, H))
    F = rng.normal(0.0, 1.0, (5, 4 * d))
    y = np.array([1.0, 0.0, 1.0, 0.0, 0.0])
    return theta, F, y


def _loss(theta, F, y, d, H, w_pos):
    z, _ = P.forward(theta, F, d, H)
    return P.bce_loss(z, y, w_pos)


@pytest.mark.parametrize("w_pos", [1.0, 2.5])
def test_backward_matches_central_differences(w_pos):
    d, H = 2, 6
    theta, F, y = _net(d, H, 3)
    z, cache = P.forward(theta, F, d, H)
    g = P.backward(theta, cache, P.bce_grad(z, y, w_pos), d, H)
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num[i] = (_loss(tp, F, y, d, H, w_pos) - _loss(tm, F, y, d, H, w_pos)) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-8 * max(1.0, np.max(np.abs(g)))
    # every block of the gradient is exercised (a dropped term would zero one)
    for blk in P.unpack(g, d, H):
        assert np.any(blk != 0)


def test_bce_grad_closed_form_and_differences():
    z = np.array([-3.0, -0.2, 0.0, 0.7, 4.0])
    y = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    w = 3.0
    g = P.bce_grad(z, y, w)
    p = 1.0 / (1.0 + np.exp(-z))
    assert np.allclose(g, (w * y * (p - 1.0) + (1.0 - y) * p) / len(z), rtol=1e-15, atol=0)
    for i in range(len(z)):
        zp, zm = z.copy(), z.copy()
        zp[i] += 1e-6
        zm[i] -= 1e-6
        assert abs((P.bce_loss(zp, y, w) - P.bce_loss(zm, y, w)) / 2e-6 - g[i]) < 1e-9


def test_only_output_bias_closed_form():
    d, H = 3, 4
    theta = np.zeros(P.param_count(d, H))
    theta[-1] = 0.3                                   # b3
    F = np.ones((4, 4 * d))
    y = np.array([1.0, 0.0, 0.0, 1.0])
    z, cache = P.forward(theta, F, d, H)
    assert np.all(z == 0.3)
    p = 1.0 / (1.0 + math.exp(-0.3))
    w = 2.0
    L = -(w * 2 * math.log(p) + 2 * math.log(1 - p)) / 4
    assert abs(P.bce_loss(z, y, w) - L) < 1e-15
    g = P.backward(theta, cache, P.bce_grad(z, y, w), d, H)
    W1, b1, W2, b2, w3, b3 = P.unpack(g, d, H)
    assert abs(b3[0] - (w * 2 * (p - 1) + 2 * p) / 4) < 1e-15
    for blk in (W1, b1, W2, b2, w3):    # every hidden unit is dead at zero weights
        assert np.all(blk == 0)


def test_hand_worked_forward():
    # d = 1, H = 2; f = [2, 1, 0, 0]
    W1 = np.array([[1.0, 0, 0, 0], [0, -1.0, 0, 0]])
    b1 = np.array([0.0, 0.5])
    W2 = np.array([[1.0, 1.0], [0.0, 2.0]])
    b2 = np.array([0.0, -1.0])
    w3 = np.array([1.0, -0.5])
    b3 = np.array([0.25])
    theta = P.pack(W1, b1, W2, b2, w3, b3)
    z, c = P.forward(theta, np.array([[2.0, 1.0, 0.0, 0.0]]), 1, 2)
    # z1 = [2, -0.5] -> h1 = [2, 0]; z2 = [2, -1] -> h2 = [2, 0]; z = 2 + 0.25
    assert list(c["h1"][0]) == [2.0, 0.0] and list(c["h2"][0]) == [2.0, 0.0]
    assert z[0] == 2.25


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = P.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01, eps=1e-8)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_generator():
    rng = np.random.Generator(np.random.PCG64(8))
    x = rng.normal(0.0, 1.0, 4096).astype(np.float32)
    x[:4] = [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0]   # ties to even
    a = P.round_bf16(x)
    b = kgsynth.bf16_bits_to_f32(kgsynth.f32_to_bf16_bits(x)).astype(np.float64)
    assert np.array_equal(a, b)
    assert a[0] == 1.0 and a[1] == 1.0 + 4 * 2.0 ** -8 and a[2] == -1.0


def test_keep_rule():
    assert P.keep_count(0, 100) == 0
    assert P.keep_count(1, 100) == 1
    assert P.keep_count(10, 100) == 1
    assert P.keep_count(11, 100) == 2
    assert P.keep_count(30, 100) == 3      # no float rounding at 10% of 30
    s = np.array([0.1, 0.9, 0.5, 0.9, 0.2, 0.3, 0.4, 0.6, 0.7, 0.8, 0.05])
    assert sorted(P.keep_top_fraction(s, 100).tolist()) == [1, 3]     # two tied at the top
    assert sorted(P.keep_top_fraction(s, 300).tolist()) == [1, 3, 8, 9]
