"""Pins of the pruner's FP64 oracle (CPU only): finite differences, closed
forms, a hand-worked forward pass, Adam's first step, the keep rule."""

import math

import numpy as np
import pytest

import kgsynth
from oracle import pruner as P
from oracle import pruner as OP


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


def _emulate_fp32(theta, F, y, w_pos, d, H, seed):
    """The bfloat16-operand network evaluated the way the kernels do it, in
    float32 with the products summed in a shuffled order (a different order
    from the FP64 reference): a stand-in GPU for checking that the
    element-wise bounds hold."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f32 = np.float32
    W1, b1, W2, b2, w3, b3 = (np.asarray(a, f32) for a in OP.unpack(theta, d, H))
    rb = lambda a: OP.round_bf16(a).astype(f32)

    def mm(A, B):   # sum over k in a random order, one float32 rounding per step
        perm = rng.permutation(A.shape[1])
        out = np.zeros((A.shape[0], B.shape[1]), f32)
        for k in perm:
            out = (out + np.outer(A[:, k], B[k, :]).astype(f32)).astype(f32)
        return out
    Fq, W1q, W2q, w3q = rb(F), rb(W1), rb(W2), rb(w3)
    z1 = (mm(Fq, W1q.T) + b1).astype(f32)
    h1 = rb(np.maximum(z1, 0))
    z2 = (mm(h1, W2q.T) + b2).astype(f32)
    h2 = rb(np.maximum(z2, 0))
    z = (mm(h2, w3q[:, None])[:, 0] + b3[0]).astype(f32)
    dz = OP.bce_grad(z.astype(np.float64), y, w_pos).astype(f32)
    g_w3 = mm(h2.T, dz[:, None])[:, 0]
    g_b3 = np.array([dz.sum(dtype=f32)], f32)
    dz2 = rb((np.outer(dz, w3q) * (z2 > 0)).astype(f32))
    g_W2 = mm(dz2.T, h1)
    g_b2 = dz2.sum(0, dtype=f32)
    dz1 = rb((mm(dz2, W2q) * (z1 > 0)).astype(f32))
    g_W1 = mm(dz1.T, Fq)
    g_b1 = dz1.sum(0, dtype=f32)
    return z.astype(np.float64), OP.pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def test_elementwise_bounds_hold_for_an_fp32_evaluation():
    """The element-wise bounds of forward_bounds / backward_bounds cover a
    float32 evaluation with another summation order (every element), and
    are not vacuous (the typical bound is far below the typical value)."""
    d, H, N = 8, 32, 96
    rng = np.random.Generator(np.random.PCG64(21))
    theta = rng.normal(0, 1, OP.param_count(d, H))
    W1, b1, W2, b2, w3, b3 = OP.unpack(theta, d, H)
    W1 *= 2 / np.sqrt(4 * d); W2 *= 2 / np.sqrt(H); w3 *= 1 / np.sqrt(H); b1 *= 0.1; b2 *= 0.1
    theta = theta.astype(np.float32).astype(np.float64)
    F = rng.normal(0, 1 / np.sqrt(d), (N, 4 * d)).astype(np.float32).astype(np.float64)
    y = (rng.random(N) < 0.3).astype(np.float64)
    z, e_z, cache = OP.forward_bounds(theta, F, d, H)
    g, e_g = OP.backward_bounds(theta, cache, z, e_z, y, 2.0, d, H)
    for seed in (1, 2, 3):
        z32, g32 = _emulate_fp32(theta, F, y, 2.0, d, H, seed)
        assert np.all(np.abs(z32 - z) <= e_z), np.max(np.abs(z32 - z) - e_z)
        assert np.all(np.abs(g32 - g) <= e_g + 1e-30)
    assert np.median(e_z / (np.abs(z) + 1e-30)) < 0.05
    nz = np.abs(g) > 0
    assert np.median(e_g[nz] / np.abs(g[nz])) < 0.05
    # a planted mistake in the reference (a dropped bias) breaks the check
    theta_bad = theta.copy()
    OP.unpack(theta_bad, d, H)[1][:] = 0.0
    z_bad, e_bad, _ = OP.forward_bounds(theta_bad, F, d, H)
    z32, _ = _emulate_fp32(theta, F, y, 2.0, d, H, 1)
    assert np.any(np.abs(z32 - z_bad) > e_bad)


def test_quantum_is_the_largest_power_of_two_divisor():
    q = OP.quantum(np.array([0.75, 3.0, -1.5 * 2.0 ** -10, 2.0 ** -126, 1.0 + 2.0 ** -23, 0.0]))
    assert q[:5].tolist() == [0.25, 1.0, 2.0 ** -11, 2.0 ** -126, 2.0 ** -23]
    assert np.isinf(q[5])


def test_grid_valued_network_is_exact_and_gradient_bounds_hold():
    """Weights and features on power-of-two grids with small integer
    multiples: every forward sum is provably exact (bound zero), a float32
    evaluation in a shuffled order reproduces the FP64 logits bit for bit,
    and the backward bounds hold element by element and stay tight.  A
    planted mistake (a bias left out of the reference) breaks the equality."""
    d, H, N = 8, 32, 96
    rng = np.random.Generator(np.random.PCG64(23))
    W1 = kgsynth.grid_values(rng, (H, 4 * d), 1, -5, 0.5)
    b1 = kgsynth.grid_values(rng, H, 4, -8)
    W2 = kgsynth.grid_values(rng, (H, H), 1, -4, 0.5)
    b2 = kgsynth.grid_values(rng, H, 4, -12)
    w3 = np.ldexp(rng.choice([-1.0, 1.0], H), -4)
    theta = OP.pack(W1, b1, W2, b2, w3, np.array([np.ldexp(3.0, -16)]))
    F = kgsynth.grid_values(rng, (N, 4 * d), 2, -3)
    y = (rng.random(N) < 0.3).astype(np.float64)
    z, e_z, cache = OP.forward_bounds(theta, F, d, H)
    assert np.all(e_z == 0) and np.all(cache["e_h1"] == 0) and np.all(cache["e_z2"] == 0)
    g, e_g = OP.backward_bounds(theta, cache, z, e_z, y, 2.0, d, H)
    for seed in (1, 2):
        z32, g32 = _emulate_fp32(theta, F, y, 2.0, d, H, seed)
        assert np.array_equal(z32, z)
        assert np.all(np.abs(g32 - g) <= e_g + 1e-30)
    nz = np.abs(g) > 0
    assert np.median(e_g[nz] / np.abs(g[nz])) < 0.02
    bad = theta.copy()
    OP.unpack(bad, d, H)[3][:] = 0.0
    assert not np.array_equal(OP.forward_bounds(bad, F, d, H)[0], z32)


def _adam_fp32(theta, g, m, v, step, lr, b1, b2, eps):
    """The Adam update in float32 operations, as the device evaluates it."""
    f = np.float32
    theta, g, m, v = (np.asarray(a, f) for a in (theta, g, m, v))
    lr, b1, b2, eps = f(lr), f(b1), f(b2), f(eps)
    bc1 = f(1) - np.power(b1, f(step), dtype=f)
    bc2 = f(1) - np.power(b2, f(step), dtype=f)
    m1 = b1 * m + (f(1) - b1) * g
    v1 = b2 * v + (f(1) - b2) * g * g
    th = theta - lr * (m1 / bc1) / (np.sqrt(v1 / bc2) + eps)
    return th.astype(np.float64), m1.astype(np.float64), v1.astype(np.float64)


def test_adam_interval_contains_fp32_updates():
    """adam_interval holds the float32 update for gradients anywhere in the
    interval, holds the FP64 update, is narrow where the gradient is
    known tightly, and excludes an update that skips the bias correction."""
    rng = np.random.Generator(np.random.PCG64(31))
    n = 20000
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    b1, b2, eps, lr = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8, 1e-3))
    theta = f32(rng.normal(0, 0.1, n))
    g = f32(rng.normal(0, 1e-3, n) * np.exp(rng.normal(0, 2, n)))
    e_g = np.abs(g) * 10.0 ** rng.uniform(-6, -2, n)
    for step, m, v in [(1, np.zeros(n), np.zeros(n)),
                       (6, f32(rng.normal(0, 1e-3, n)), f32(rng.random(n) * 1e-5))]:
        (tlo, thi), (mlo, mhi), (vlo, vhi) = OP.adam_interval(theta, g, e_g, m, v, step, lr, b1, b2, eps)
        for frac in (-1.0, -0.3, 0.0, 0.7, 1.0):
            gg = f32(g + frac * e_g * 0.9)
            inside = np.abs(gg - g) <= e_g          # float32 rounding may leave the interval
            assert np.mean(inside) > 0.99
            th, m1, v1 = _adam_fp32(theta, gg, m, v, step, lr, b1, b2, eps)
            assert np.all(((tlo <= th) & (th <= thi))[inside])
            assert np.all(((mlo <= m1) & (m1 <= mhi))[inside]) and np.all(((vlo <= v1) & (v1 <= vhi))[inside])
        t64, _, _ = OP.adam_step(theta, g, m, v, step, lr, b1, b2, eps)
        assert np.all((tlo <= t64) & (t64 <= thi))
        tight = e_g < 1e-5 * np.abs(g)
        assert np.median(((thi - tlo) / (lr * 1e-3 + np.abs(t64 - theta)))[tight]) < 1e-3
        # no bias correction: outside the interval for most elements
        th_bad = theta - lr * (b1 * m + (1 - b1) * g) / (np.sqrt(b2 * v + (1 - b2) * g * g) + eps)
        assert np.mean((th_bad < tlo) | (th_bad > thi)) > 0.9
