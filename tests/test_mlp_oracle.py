"""Pins of the surrogate network's FP64 oracle (oracle/mlp.py) against values
fixed by the mathematics: hand-rounded bfloat16 values, the normal CDF,
finite differences, Adam's closed form and a one-hot network."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp
from workloads.surrogate import LAYERS, c5_features, init_ensemble, init_member, n_params

SMALL = (5, 7, 6, 4, 3)


def bf16_bits(x32):
    """float32 -> bfloat16 by rounding the bit pattern (ties to even)."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_hand_values():
    cases = {1.0: 1.0, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6, 1 + 2 ** -7: 1 + 2 ** -7,
             math.pi: 3.140625, -0.1: -0.10009765625, 0.0: 0.0, 2 ** -20 * 1.00390625: 2 ** -20,
             255.5: 256.0, 254.5: 254.0, -1e30: -202 * 2.0 ** 92}   # 1e30 = 1.5777 * 2^99 -> 202 / 128 * 2^99
    for x, want in cases.items():
        assert mlp.bf16(x) == want, (x, mlp.bf16(x), want)


def test_bf16_matches_bit_rounding_of_float32():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), bf16_bits(x))


def test_gelu_matches_normal_cdf():
    z = np.linspace(-6, 6, 1001)
    assert np.abs(mlp.gelu(z) - z * norm.cdf(z)).max() < 1e-15
    assert mlp.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, abs=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(mlp.gelu_grad(z) - fd).max() < 1e-8


def test_layout_one_hot_network():
    """z_o = sum_i W[o][i] a_i + b_o: a path through single weights picks
    input 3 -> hidden 5 -> hidden 1 -> hidden 2 -> output 0."""
    parts = []
    path = [(5, 3), (1, 5), (2, 1), (0, 2)]
    for (i, o), (po, pi) in zip(zip(SMALL[:-1], SMALL[1:]), path):
        W = np.zeros((o, i))
        W[po, pi] = 1.0
        parts.append((W, np.zeros(o)))
    theta = mlp.pack(parts)
    X = np.zeros((2, SMALL[0]))
    X[0, 3] = 2.0
    X[1, 4] = 2.0
    out, _ = mlp.forward(theta, X, mixed=False, layers=SMALL)
    g3 = mlp.gelu(mlp.gelu(mlp.gelu(2.0)))
    assert out[0, 0] == pytest.approx(g3, abs=1e-15)
    assert np.abs(out[0, 1:]).max() == 0 and np.abs(out[1]).max() == 0


def test_gradient_matches_finite_differences_small():
    rng = np.random.default_rng(1)
    n = sum(o * i + o for i, o in zip(SMALL[:-1], SMALL[1:]))
    theta = rng.standard_normal(n) * 0.7
    X = rng.uniform(0, 1, (6, SMALL[0]))
    Y = rng.standard_normal((6, SMALL[-1]))
    _, g = mlp.loss_and_grad(theta, X, Y, mixed=False, layers=SMALL)
    h = 1e-6
    fd = np.empty(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        lp, _ = mlp.loss_and_grad(theta + e, X, Y, mixed=False, layers=SMALL)
        lm, _ = mlp.loss_and_grad(theta - e, X, Y, mixed=False, layers=SMALL)
        fd[k] = (lp - lm) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_gradient_matches_finite_differences_full_network_sample():
    theta = init_member(7).astype(np.float64)
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, (4, 24))
    Y = rng.uniform(-1, 1, (4, 10))
    _, g = mlp.loss_and_grad(theta, X, Y, mixed=False)
    # coordinates from every weight matrix and bias vector
    bounds = np.cumsum([0] + [s for i, o in zip(LAYERS[:-1], LAYERS[1:]) for s in (o * i, o)])
    idx = np.concatenate([rng.integers(lo, hi, 12) for lo, hi in zip(bounds[:-1], bounds[1:])])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss_and_grad(theta + e, X, Y, mixed=False)[0] -
              mlp.loss_and_grad(theta - e, X, Y, mixed=False)[0]) / (2 * h)
        assert abs(g[k] - fd) <= 1e-8 + 1e-6 * abs(fd), (k, g[k], fd)


def test_mixed_precision_gradient_close_to_fp64():
    theta = init_member(8).astype(np.float64)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (64, 24))
    Y = rng.uniform(-1, 1, (64, 10))
    l0, g0 = mlp.loss_and_grad(theta, X, Y, mixed=False)
    l1, g1 = mlp.loss_and_grad(theta, X, Y, mixed=True)
    assert abs(l1 - l0) <= 2e-2 * l0
    assert np.linalg.norm(g1 - g0) <= 3e-2 * np.linalg.norm(g0)
    # the rounding is really applied: results differ
    assert np.abs(g1 - g0).max() > 0


def test_adam_closed_form_constant_gradient():
    rng = np.random.default_rng(4)
    theta0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    th = theta0
    lr, eps = 1e-3, 1e-8
    for t in range(1, 8):
        th, m, v = mlp.adam(th, m, v, g, t, lr, eps=eps)
    assert np.abs(th - (theta0 - 7 * lr * g / (np.abs(g) + eps))).max() < 1e-12


def test_ensemble_spread_is_population_std():
    thetas = init_ensemble(seed=11).astype(np.float64)
    X = np.random.default_rng(5).uniform(0, 1, (9, 24))
    mean, spread, P = mlp.ensemble(thetas, X)
    assert np.allclose(mean, P.mean(axis=0), atol=0, rtol=0)
    assert np.allclose(spread, np.std(P, axis=0, ddof=0).max(axis=1), rtol=1e-14, atol=0)
    # hand example: members 0, 0, 0, 1 -> std sqrt(3)/4
    Q = np.array([0.0, 0.0, 0.0, 1.0])
    assert np.sqrt(((Q - Q.mean()) ** 2).mean()) == pytest.approx(math.sqrt(3) / 4, abs=1e-16)


def test_training_reduces_loss_on_a_smooth_target():
    """A few Adam steps on the oracle lower the loss of a smooth regression."""
    rng = np.random.default_rng(6)
    theta = init_member(9).astype(np.float64)
    X = rng.uniform(0, 1, (64, 24))
    Y = np.cos(2 * np.pi * X[:, :10]) * 0.5
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, X, Y)[0]
    for t in range(1, 31):
        _, g = mlp.loss_and_grad(theta, X, Y)
        theta, m, v = mlp.adam(theta, m, v, g, t, 1e-3)
    assert mlp.loss_and_grad(theta, X, Y)[0] < 0.75 * l0


def test_feature_scaling_and_init_shapes():
    from workloads import c5_draw_samples
    dev, ang = c5_draw_samples(1000, seed=12)
    F = c5_features(dev, ang)
    assert F.shape == (1000, 24) and F.dtype == np.float32
    assert F.min() >= 0 and F.max() <= 1
    W = init_ensemble()
    assert W.shape == (4, n_params()) and n_params() == 140554
